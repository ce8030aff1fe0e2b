/*
 * lq.h -- C ABI of the MI355X (gfx950) Wilson / Wilson-clover fermion-matrix
 * library: the fermion matrix of eq. (1), Sec. 3 of Akahoshi et al.,
 * "General purpose lattice QCD code set Bridge++ 2.0 for high performance
 * computing" (arXiv:2111.04457), its even-odd Schur form, and the Krylov
 * solvers that compute quark propagators with it (Sec. 2, Fig. 1).
 *
 * The calls follow the usage of the paper's Fig. 1: an operator object is
 * created from fermion parameters (params_fopr), given a gauge field
 * (set_config), applied in a mode (set_mode: D, Ddag, DdagD, ...), and
 * inverted to a tolerance with a mixed-precision solver (invert(x, b, nconv,
 * diff)).
 *
 * Conventions shared by every call
 * --------------------------------
 *  dims      (Lx, Ly, Lz, Lt), each even and >= 2.  V = Lx Ly Lz Lt.
 *  lex site  x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2 (even = 0).
 *  gauge     complex128 U[t][z][y][x][mu][a][b], mu = 0..3 for x, y, z, t;
 *            (U psi)_a = sum_b U_ab psi_b.  Links must be SU(3) when 12-real
 *            compression is used.
 *  spinor    full field: complex128 [V][4 spin][3 colour] in lex order
 *            (spin-colour index ic + 3*is, as in Fig. 1);
 *            parity field: complex128 [V/2][4][3] in checkerboard order
 *            cb = lex / 2 (integer division), holding the sites of one parity.
 *            Several right-hand sides are stacked on a leading axis [nrhs].
 *  gamma     chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
 *            gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1).
 *  boundary  a hop x -> x+mu across the lattice edge is multiplied by the
 *            phase bc[mu] (|bc| = 1); the backward hop by its conjugate
 *            (the paper: a boundary condition imposed in each direction).
 *  clover    F(x) = -c_sw kappa sum_{mu<nu} gamma_mu gamma_nu (x) Fhat_{mu nu}(x),
 *            Fhat = (Q - Q^dag)/8 of the four counter-clockwise plaquettes Q
 *            at x (colour trace removed unless clover_traceless = 0).  In
 *            the chiral basis A = 1 + F is two 6x6 Hermitian blocks.
 *  even-odd  D = [[A_ee, -kappa H_eo], [-kappa H_oe, A_oo]] with H the
 *            hopping sum of eq. (1); Schur operator
 *            M = A_ee - kappa^2 H_eo A_oo^-1 H_oe on even sites.
 *
 * Memory and streams
 * ------------------
 *  Every spinor / gauge pointer is a DEVICE pointer owned by the caller and
 *  borrowed for the duration of the call, except in the *_host variants
 *  (lq_op_set_gauge_host, lq_op_apply_host, lq_solve_host), which take host
 *  pointers and stage them through device buffers of the operator.
 *  The operator's device memory (packed links and clover in every
 *  precision, the packed fields and work vectors of applies and solves) is
 *  either one workspace the caller allocates and binds (lq_op_bind; its
 *  size from lq_op_workspace_bytes), so that set_gauge, set_params, apply
 *  and solve allocate nothing, or, unbound, allocated by the library on
 *  first use (lq_op_set_gauge, the first apply or solve of a size) and
 *  freed by lq_op_destroy.  The force, molecular-dynamics, eigensolver,
 *  deflation and tuner calls and lq_field_create allocate their own extra
 *  buffers in either case.  `stream` is a hipStream_t (NULL = the default
 *  stream); every call is ordered on it.  Calls that return host results
 *  (solves, forces, norms, host variants) synchronize the stream.
 *  An lq_op is not thread-safe: calls on one lq_op must not overlap.
 *
 * Errors
 * ------
 *  Every call returns an lq_status.  Negative values are errors (outputs
 *  unspecified); LQ_NOT_CONVERGED (+1) means the solution, nconv and diff
 *  were still filled.  Arguments are validated on the host before any
 *  device work.  lq_last_error() returns a message for the calling thread's
 *  last failure.
 */
#ifndef LQ_H
#define LQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lq_op lq_op;
typedef struct lq_field lq_field;
typedef struct lq_batch lq_batch;
typedef struct lq_mg lq_mg;

typedef enum {
    LQ_OK = 0,
    LQ_NOT_CONVERGED = 1,
    LQ_ERR_ARG = -1,
    LQ_ERR_STATE = -2,
    LQ_ERR_HIP = -3,
    LQ_ERR_NOMEM = -4,
    LQ_ERR_SINGULAR = -5,
    LQ_ERR_NONFINITE = -6,
    LQ_ERR_NODEVICE = -7
} lq_status;

/* Storage precision of packed fields.  LQ_F16 stores links as IEEE binary16
 * and spinors as binary16 with one FP32 scale per site; arithmetic is FP32. */
typedef enum { LQ_F64 = 0, LQ_F32 = 1, LQ_F16 = 2 } lq_prec;

/* Operator kinds (the set_mode analogue of Fig. 1).
 * Full-lattice kinds act on full fields, the others on parity fields. */
typedef enum {
    LQ_D = 0,             /* D of eq. (1)                          full */
    LQ_DDAG = 1,          /* D^dag                                 full */
    LQ_DDAGD = 2,         /* D^dag D                               full */
    LQ_SCHUR = 3,         /* M = A_ee - kappa^2 H_eo A_oo^-1 H_oe   even -> even */
    LQ_SCHUR_DAG = 4,     /* M^dag                                 even -> even */
    LQ_SCHUR_NORMAL = 5,  /* M^dag M                               even -> even */
    LQ_HOP_EO = 6,        /* H_eo (odd -> even)                    */
    LQ_HOP_OE = 7,        /* H_oe (even -> odd)                    */
    LQ_HOP_EO_DAG = 8,    /* (H_oe)^dag (odd -> even)              */
    LQ_HOP_OE_DAG = 9,    /* (H_eo)^dag (even -> odd)              */
    LQ_CLOVER_E = 10,     /* A_ee                                  even -> even */
    LQ_CLOVER_O = 11,     /* A_oo                                  odd -> odd */
    LQ_CLOVER_INV_O = 12, /* A_oo^-1                               odd -> odd */
    LQ_SCHUR_LEFT = 13    /* A_ee^-1 M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe  even -> even */
} lq_kind;

typedef enum { LQ_CGNE = 0, LQ_BICGSTAB = 1 } lq_solver_kind;

/* Fermion parameters (params_fopr of Fig. 1). */
typedef struct {
    int dims[4];          /* Lx, Ly, Lz, Lt: even, >= 2 */
    double kappa;         /* hopping parameter, kappa = 1/(8 + 2 m0); finite */
    double csw;           /* clover coefficient; 0 = Wilson (F = 0) */
    double bc[4][2];      /* boundary phase per direction as (re, im), |phase| = 1 */
    int clover_traceless; /* 1 (default): colour trace of Fhat removed */
    int link_recon;       /* 18 or 12: reals per link read by the hopping kernels (all
                             precisions; 12 stores rows 0 and 1 and rebuilds row 2 as
                             conj(row0 x row1), valid for SU(3) links only) */
    double twist;         /* twisted-mass Wilson operator D = 1 - kappa H + i twist gamma_5
                             (twist = 2 kappa mu for a twisted mass mu); 0 (default): none.
                             Finite; not with the clover term (csw must be 0).  D^dag of a
                             twisted operator is gamma_5 D(-twist) gamma_5: the modes
                             LQ_DDAG and LQ_DDAGD solve with the sign of twist flipped
                             for the duration of the call (deflate = 1 needs LQ_D) */
} lq_op_params;

/* Solver parameters (params_solver of Fig. 1). */
typedef struct {
    int solver;           /* lq_solver_kind */
    double tol;           /* target true relative residual |b - D x| / |b| (FP64) */
    int max_iter;         /* cap on total inner Krylov iterations */
    int inner;            /* lq_prec of the inner solve; LQ_F64 = plain FP64 solve */
    double inner_tol;     /* residual reduction asked of each inner solve (mixed) */
    int max_outer;        /* cap on FP64 defect-correction steps */
    int check_every;      /* inner iterations between host convergence checks */
    int even_odd;         /* 1: solve the Schur system (default); 0: full lattice (CGNE only) */
    int left_precond;     /* 1: each inner BiCGStab solve of the even-odd system runs on
                             A_ee^-1 M with the source A_ee^-1 r (clover only; the outer
                             FP64 loop keeps the residual of M x = b); default 0 */
    int reliable;         /* 1: reliable updates -- after each FP64 residual replacement the
                             inner Krylov solver continues its search directions (CG: p,
                             BiCGStab: p, v and the shadow residual) on the new residual
                             instead of starting a new space; a system whose last inner
                             solve broke down, stopped at the iteration cap or made no
                             iteration starts afresh.  0 (default): each inner solve
                             starts from scratch (plain defect correction) */
    int deflate;          /* 1: before each inner solve the outer loop projects the FP64
                             residual with the operator's deflation space
                             (lq_op_set_deflation): x += sum_k v_k v_k^dag M^dag r / lambda_k,
                             r -= M of that (for M^dag M x = b: v_k^dag r and M^dag M).
                             Even-odd solves of one operator (not lq_batch_solve); an
                             operator without a deflation space is LQ_ERR_STATE.  0
                             (default): no deflation */
} lq_solver_params;

/* Per-system solve statistics (nconv and diff of Fig. 1's invert). */
typedef struct {
    int nconv;            /* total inner Krylov iterations */
    int nouter;           /* FP64 defect-correction steps */
    int restarts;         /* Krylov restarts after breakdown */
    int converged;        /* 1 if diff <= tol */
    double diff;          /* true residual |b - D x|_2 / |b|_2 in FP64 (not squared), recomputed
                             from the final x (not the Krylov recursion); for the even-odd
                             solve as |b_e + kappa H_eo A_oo^-1 b_o - M x_e|, equal to it since
                             the reconstructed x_o satisfies the odd rows exactly */
    double t_solve_ms;    /* wall time of the solve (all systems of the call together) */
    double hop_bytes;     /* algorithmic bytes of the hopping-term applies of the call
                             (lq_op_traffic per apply), all systems together */
    int n_hop;            /* parity hopping-term applies of the call, all precisions */
} lq_solve_stats;

/* Defaults: lq_op_params with kappa = 0.125, csw = 0, periodic phases,
 * traceless clover, 18-real links; lq_solver_params with BiCGStab,
 * tol 1e-10, FP32 inner, inner_tol 1e-5, even-odd. */
void lq_op_params_default(lq_op_params *p);
void lq_solver_params_default(lq_solver_params *p);

/* Version string of the library. */
const char *lq_version(void);

/* Message describing the calling thread's last error ("" if none). */
const char *lq_last_error(void);

/* Create an operator for the parameters (validated on the host: even dims
 * >= 2, finite kappa and csw, |bc| = 1, link_recon in {12, 18}).  No device
 * memory is allocated here (only a stream and two events are created).
 * LQ_ERR_NODEVICE if no gfx950 device is visible. */
lq_status lq_op_create(const lq_op_params *p, lq_op **out);
void lq_op_destroy(lq_op *op);

/* Device memory (the interface object of Sec. 3.3 that holds the fields in
 * the device layout; params_fopr / set_config / invert of Fig. 1 then run
 * on it).
 * lq_workspace_bytes: bytes of the workspace of an operator with parameters
 * p for calls of up to nrhs right-hand sides: the packed links (FP64 with
 * 18 reals; FP32, FP16 and, with link_recon 12, FP64 with link_recon
 * reals), the clover blocks A and A^-1 in three precisions (csw != 0 only),
 * the packed fields of an apply and of a solve, the staging of host fields,
 * the reduction partials, the solver scalars and the solver's vectors, each
 * region starting on a 256-byte boundary.  Host arithmetic only: no device
 * is needed.  LQ_ERR_ARG for invalid dims, link_recon or nrhs < 1.
 * lq_op_workspace_bytes: the same for an existing operator (its current
 * csw decides whether clover blocks are stored). */
lq_status lq_workspace_bytes(const lq_op_params *p, int nrhs, size_t *bytes);
lq_status lq_op_workspace_bytes(const lq_op *op, int nrhs, size_t *bytes);

/* Bind dev_mem (a device allocation of `bytes` bytes on the operator's
 * device, owned by the caller, e.g. a torch uint8 tensor, 256-byte aligned)
 * as the operator's device memory; it must stay allocated until the
 * operator is destroyed or bound again.  The layout is that of
 * lq_op_workspace_bytes for the largest nrhs whose size fits in `bytes`
 * (lq_op_get_option "bound_nrhs"); calls with more right-hand sides return
 * LQ_ERR_ARG.  Binding drops the gauge field (call lq_op_set_gauge again)
 * and frees what the library had allocated; dev_mem = NULL unbinds (the
 * library allocates on demand again).  Waits for the device to be idle.
 * After binding, lq_op_set_gauge, lq_op_set_params, lq_op_apply,
 * lq_op_apply_field and lq_solve (and their host variants) allocate no
 * device memory ("owned_kib" stays 0); setting csw != 0 on an operator bound
 * with csw = 0 returns LQ_ERR_NOMEM (no room for the clover blocks).
 * LQ_ERR_ARG if bytes is below lq_op_workspace_bytes(op, 1) or dev_mem is
 * misaligned. */
lq_status lq_op_bind(lq_op *op, void *dev_mem, size_t bytes);

/* Set the gauge field (set_config of Fig. 1).  U: device complex128 in the
 * gauge layout.  Packs FP64, FP32 and FP16 copies (even/odd split, SoA),
 * builds A = 1 + F and A_oo^-1 in FP64 and down-converts them.
 * LQ_ERR_SINGULAR if a clover block of an odd site is not invertible
 * (A_oo is the block the even-odd solve inverts; A_ee is only applied). */
lq_status lq_op_set_gauge(lq_op *op, const void *U, void *stream);
/* The same with U in host memory (copied to the operator's device memory
 * on the stream first; synchronizes it). */
lq_status lq_op_set_gauge_host(lq_op *op, const void *U, void *stream);

/* Change kappa, csw and the boundary phases; rebuilds the clover term from
 * the stored links.  bc may be NULL to keep the phases. */
lq_status lq_op_set_params(lq_op *op, double kappa, double csw, const double bc[4][2], void *stream);

/* out = K in for kind K with packed storage/arithmetic precision prec.
 * in, out: device complex128 in the full or parity spinor layout of K,
 * nrhs right-hand sides stacked; in != out.  Full-lattice kinds use FP64
 * only at the boundary; prec selects the internal precision. */
lq_status lq_op_apply(lq_op *op, lq_kind kind, lq_prec prec, void *out, const void *in, int nrhs,
                      void *stream);
/* The same with in and out in host memory (staged through device buffers of
 * the operator; the same kernels, so the same bits; synchronizes the
 * stream). */
lq_status lq_op_apply_host(lq_op *op, lq_kind kind, lq_prec prec, void *out, const void *in, int nrhs,
                           void *stream);

/* lq_op_apply without any device allocation, for callers that cannot
 * allocate: code being captured into a HIP graph, tight serving loops,
 * hosts that forbid hipMalloc.  Same arguments, kinds and results as
 * lq_op_apply (the same kernels run, so the outputs are the same bits); the
 * packed copies of in and out and the temporaries of the composite kinds
 * live in a fixed 64 MiB device array inside the library (one per GPU, held
 * until the process ends), not in memory the call allocates.
 * Limit: the packed fields must fit in 64 MiB, i.e.
 *   2 F + T <= 64 MiB,  F = (full kind ? 2 : 1) * nrhs * V/2 * s,
 *   T = nrhs * V/2 * s for LQ_SCHUR, LQ_SCHUR_DAG and LQ_SCHUR_LEFT, 2 nrhs V/2 s
 *   for LQ_SCHUR_NORMAL and LQ_DDAGD, else 0, with s = 192, 96 or 52 bytes for
 *   FP64, FP32 and FP16 (V/2 rounded up to a multiple of 64, each part to
 *   256 bytes); larger calls return LQ_ERR_ARG before any device work (e.g.
 *   16^3 x 32 fits every kind in FP64 with nrhs = 1).
 * Every call on one GPU shares that array: calls that overlap in time on the
 * same GPU (other streams, other threads, other operators) race and must be
 * ordered by the caller.  No part of the array needs to start at zero.
 * LQ_SCHUR_LEFT computes A_ee^-1 on its first use after a gauge update
 * (allocation-free, but it synchronizes the stream). */
lq_status lq_op_apply_noalloc(lq_op *op, lq_kind kind, lq_prec prec, void *out, const void *in, int nrhs,
                              void *stream);

/* Device-resident parity spinor fields in the library's packed layout
 * (structure of arrays over checkerboard sites, nrhs stacked), for applying
 * kinds >= LQ_SCHUR without packing at every call. */
lq_status lq_field_create(lq_op *op, lq_prec prec, int nrhs, lq_field **out);
void lq_field_destroy(lq_field *f);
/* Import from / export to a device complex128 parity field [nrhs][V/2][4][3]. */
lq_status lq_field_import(lq_field *f, const void *src, void *stream);
lq_status lq_field_export(const lq_field *f, void *dst, void *stream);
/* out = K in on packed fields of the same precision and nrhs (K >= LQ_SCHUR). */
lq_status lq_op_apply_field(lq_op *op, lq_kind kind, lq_field *out, const lq_field *in, void *stream);

/* Workgroup size (64 (default), 128 or 256 threads) of the hopping kernels of
 * precision prec on this operator.  The result does not depend on it: every
 * site is summed in the same order whatever the launch shape. */
lq_status lq_op_set_block(lq_op *op, lq_prec prec, int block);

/* Other execution options (none changes a result bit):
 *   "xcd_remap" -1|0|1|2  order of the hopping kernel's workgroups: 0 plain,
 *                    1 XCD-aware (each XCD takes a contiguous range of site
 *                    blocks), 2 XCD-aware with the blocks of neighbouring
 *                    time slices visited one after another (used when a time
 *                    slice of one parity is a whole number of workgroups,
 *                    else as 1); -1 (default) automatic: 0 for one
 *                    right-hand side, 2 for several (measured: plain order is
 *                    fastest alone and 15-45 % slower with several); all
 *                    precisions; "xcd_remap_f64" / "_f32" / "_f16" per precision;
 *   "graphs"    0|1  capture the solvers' inner-iteration chunks in hipGraphs (default 1);
 *   "tune_form" 0|1  the operator form lq_tune times: 0 M (default), 1 A_ee^-1 M
 *                    (clover operators; as 0 without clover);
 *   "break_at"  k>=0 the next lq_solve's first inner BiCGStab solve takes rho = 0 at
 *                    its iteration k (a forced breakdown, to exercise the restart
 *                    path: the system freezes, the FP64 outer loop restarts the
 *                    inner solve from the current iterate and counts a restart);
 *                    reset to 0 by that solve; 0 (default) never;
 *   "log_level" 0|1|2  progress lines of solves on stderr: 1 one per solve (outer
 *                    steps, iterations, restarts, residual), 2 also one per outer
 *                    step; the environment variable LQ_LOG_LEVEL sets a floor;
 *   "rhs_per_thread" 0|1|2|4  how the hopping kernel shares links between
 *                    right-hand sides applied together (0, the default:
 *                    automatic: 4 with at least 4 right-hand sides, 2 in
 *                    FP16 with 2 or 3, else 1): 1 one per thread, the
 *                    right-hand sides of one site block in adjacent
 *                    workgroups sharing the links through the L2; 2 two per
 *                    thread (each loaded link used for both; not with the
 *                    fused dot products, where 1 is used); 4 four per
 *                    workgroup of 64 sites, one wavefront each, the links
 *                    staged once in LDS, and the clover blocks too in FP16
 *                    and FP32 storage (with at least 4 right-hand sides,
 *                    else 1);
 *                    per precision "rhs_per_thread_f64" / "_f32" / "_f16".
 * lq_op_get_option also reads "hop_block_f64", "hop_block_f32", "hop_block_f16", and
 * "work_kib": the KiB of device work buffers the operator holds (temporaries,
 * reduction partials, solver, force, eigensolver and molecular-dynamics
 * workspaces; not the packed links and clover), "owned_kib": the KiB of
 * device memory the library allocated itself for the operator (0 for the
 * regions of a bound workspace), "bound_nrhs": the right-hand sides the
 * bound workspace is laid out for (0: not bound).
 * LQ_ERR_ARG for an unknown name or value. */
lq_status lq_op_set_option(lq_op *op, const char *name, int value);
lq_status lq_op_get_option(const lq_op *op, const char *name, int *value);

/* Algorithmic HBM bytes and flops of one parity hopping-term apply per
 * output site and right-hand side for the given precision, with (clover = 1)
 * or without the fused clover epilogue: compulsory traffic only (8 links,
 * one input and one output spinor, clover block if used). */
lq_status lq_op_traffic(const lq_op *op, lq_prec prec, int nrhs, int clover, double *bytes_per_site,
                        double *flops_per_site);

/* LQ_DDAGD solves D^dag y = b to tol / 2, then D x = y to tol |b| / (2 |D| |y|)
 * (|D| bounded by 1 + |twist| + 16 kappa + 12 |c_sw| kappa), so that the normal residual
 * |b - D^dag D x| / |b| reported in diff meets tol; it starts from zero
 * (use_x0 = 1 is LQ_ERR_ARG). */
/* Solve op x = b for mode LQ_D, LQ_DDAG or LQ_DDAGD (invert of Fig. 1) for
 * nrhs right-hand sides at once (multi-RHS kernels reuse every loaded link
 * across the right-hand sides).  b, x: device complex128 full fields
 * [nrhs][V][4][3]; x is the initial guess if use_x0, and is overwritten by
 * the solution.  stats: host array of nrhs entries (may be NULL).
 * Returns LQ_OK, LQ_NOT_CONVERGED (x and stats filled), or an error;
 * LQ_ERR_NONFINITE if b or an intermediate residual is not finite. */
lq_status lq_solve(lq_op *op, const lq_solver_params *sp, lq_kind mode, int nrhs, void *x, const void *b,
                   int use_x0, lq_solve_stats *stats, void *stream);
/* The same with b and x in host memory (copied through device buffers of the
 * operator; the solve itself is that of lq_solve, so x is the same bits). */
lq_status lq_solve_host(lq_op *op, const lq_solver_params *sp, lq_kind mode, int nrhs, void *x, const void *b,
                        int use_x0, lq_solve_stats *stats, void *stream);

/* Batched solve over several lattices (a ragged batch: operators of
 * different volumes and gauge fields, nrhs[i] right-hand sides each).
 * lq_batch_create validates (distinct operators on one device, nrhs >= 1)
 * and keeps the list; the operators must outlive the batch.
 * lq_batch_solve solves D_i x_i = b_i for every lattice with the same
 * solver parameters: b[i], x[i] are device complex128 full fields
 * [nrhs[i]][V_i][4][3]; stats receives sum(nrhs) entries in batch order.
 * Each lattice's solve runs on its operator's stream from a host thread of
 * its own, so the lattices' kernels overlap on the GPU; each is the same
 * solve as lq_solve (its inner iterations replayed from hipGraphs), and the
 * results equal those of separate lq_solve calls bit for bit.  On failure
 * the status and message of the first failing lattice in batch order are
 * returned (the other lattices' results are then unspecified). */
lq_status lq_batch_create(lq_op *const *ops, int nops, const int *nrhs, lq_batch **out);
lq_status lq_batch_solve(lq_batch *batch, const lq_solver_params *sp, void *const *x, const void *const *b,
                         lq_solve_stats *stats, void *stream);
void lq_batch_destroy(lq_batch *batch);

/* Autotuner: for each storage precision, times the operator work of one
 * BiCGStab iteration (two applies of the Schur operator M, or with the
 * option "tune_form" = 1 of the A_ee^-1-preconditioned form the inner solves
 * use with left_precond; the second kernel of each apply with the dot
 * products the solver fuses into it; nrhs right-hand sides) with HIP events
 * over workgroup sizes {64, 128, 256}, the three workgroup orders and, for
 * nrhs >= 4 in FP16 / FP32, four right-hand sides per workgroup sharing
 * links in LDS; requires every candidate's output to be bitwise equal to
 * the first's, and keeps the fastest on the operator unless the shape the
 * operator had is within 2 % of it (a shape that beats it in the sweep is
 * timed against it again, in turn, before it replaces it).  Results are
 * cached in the JSON file
 * cache_path (or $LQ_TUNE_CACHE; NULL and unset: no cache), keyed by
 * operator form, precision, lattice, link format, nrhs and architecture;
 * cached entries are applied without timing.  report (may be NULL)
 * receives a JSON summary, truncated to report_len bytes.  Uses (and
 * overwrites) the operator's scratch fields; synchronizes the stream. */
lq_status lq_tune(lq_op *op, int nrhs, const char *cache_path, char *report, size_t report_len, void *stream);

/* Device bandwidth probe, the reference point of the bandwidth figures
 * (not part of the method): mode 0 copies `bytes` from src to dst, mode 1
 * reads src (dst unused; one small partial sum per workgroup is written to a
 * buffer of the call), 16 bytes per thread per step over a grid of 16
 * workgroups per compute unit, non-temporal loads and stores; one warm-up
 * launch, then reps launches between HIP events on the stream: *us receives
 * the average launch duration.  bytes: a multiple of 16; src, dst: device
 * buffers, 16-byte aligned.  Synchronizes the stream. */
lq_status lq_bandwidth_probe(int mode, void *dst, const void *src, size_t bytes, int reps, double *us, void *stream);

/* Pseudofermion action and force (molecular-dynamics force of the gauge-field
 * generation the paper's Sec. 2 describes, whose solves are the bottleneck):
 *   variant 0 (even-odd):  S = phi^dag (M^dag M)^-1 phi,  M = A_ee - kappa^2 H_eo A_oo^-1 H_oe,
 *                          phi a device complex128 parity field [V/2][4][3] on even sites;
 *   variant 1 (full):      S = phi^dag (D^dag D)^-1 phi,  phi a full field [V][4][3].
 * Wilson (csw = 0, A = 1), Wilson-clover operators (eq. (1)) and twisted-mass
 * Wilson operators (A = 1 + i twist gamma_5, independent of the links: only
 * the inverses change); the clover term enters through the derivative of its
 * leaves Q_{mu nu}(x), traceless or not as the operator was built.
 * The solve runs with sp (FP64 defect correction around sp->inner); the
 * hopping-term force kernel computes in force_prec (LQ_F64 or LQ_F32), the
 * clover part always in FP64 (on the FP64 solution).  Outputs (device
 * complex128, each may be NULL):
 *   dSdU  [V][4][3][3]  the gradient of S with respect to the link entries,
 *                       dS = Re sum conj(dSdU) dU, i.e. M^dag for the matrix M
 *                       with dS = sum Re tr(M dU) (the torch convention);
 *   G     [V][4][3][3]  the su(3) force -TA(U M), so that dS/de along
 *                       U -> exp(e X) U equals sum Re tr(G^dag X);
 *   X_out               X = (M^dag M)^-1 phi (layout of phi).
 * *S receives the action.  With clover, a workspace of 6 V 144 bytes stays
 * with the operator (freed with it). */
lq_status lq_pf_force(lq_op *op, const lq_solver_params *sp, int variant, lq_prec force_prec, const void *phi,
                      void *dSdU, void *G, void *X_out, double *S, lq_solve_stats *stats, void *stream);

/* Lowest eigenpairs of the Hermitian positive even-odd normal operator
 * A = M^dag M (M the Schur operator, kind LQ_SCHUR_NORMAL, in FP64): an
 * eigenvalue solver of the kind the paper's conclusion lists among the
 * framework's algorithms.  Thick-restart Lanczos with full
 * reorthogonalisation on B = A, or (cheb_degree d >= 1) on the Chebyshev
 * filter B = T_d(((lo + hi) - 2A) / (hi - lo)), which maps the spectrum
 * below lo to the largest values of B and [lo, hi] into [-1, 1]. */
typedef struct {
    int nev;           /* wanted eigenpairs, >= 1 */
    int m;             /* basis vectors per cycle, nev + 1 <= m <= 1024 */
    int max_restarts;  /* thick restarts after the first cycle, >= 0 */
    int cheb_degree;   /* 0: Lanczos on A; d in [1, 10000]: on T_d(L(A)) */
    double cheb_lo;    /* filter interval [lo, hi]: lo > 0 should lie above the */
    double cheb_hi;    /* wanted eigenvalues, hi at or above the largest; 0 picks each
                          from one plain Lanczos cycle of m steps (hi: 1.01 (largest
                          Ritz value + its residual bound); lo: the (nev+1)-th
                          smallest Ritz value, never below the (nev+1)-th eigenvalue) */
    double tol;        /* converged when |A x - lambda x| <= tol lambda |x| */
} lq_eig_params;

typedef struct {
    int nconv;       /* pairs that met tol */
    int restarts;    /* thick restarts performed */
    long applies;    /* applications of A (each d per application of the filter) */
    double cheb_lo;  /* the filter interval used (0, 0 without the filter) */
    double cheb_hi;
} lq_eig_stats;

/* nev 8, m 64, max_restarts 100, cheb_degree 8 with the interval picked
 * automatically (cheb_lo = cheb_hi = 0), tol 1e-8 */
void lq_eig_params_default(lq_eig_params *p);

/* v0: start vector (device complex128 [V/2][4][3], nonzero).  evals[nev]
 * receive the eigenvalue estimates x^dag A x / x^dag x of the nev Ritz
 * vectors x at the wanted end of B (ascending), resid[nev] (may be NULL)
 * the residual norms |A x - lambda x| / |x| computed on the GPU, evecs (may
 * be NULL; device complex128 [nev][V/2][4][3]) the unit Ritz vectors, stats
 * (may be NULL) the counts above.  A workspace of about (2m + 2) V/2 192
 * bytes plus four packed fields (and two pinned host doubles) stays with
 * the operator: grown when a call needs more, reused by later calls, freed
 * with the operator (counted in the "work_kib" option).  When the Krylov space of v0 is invariant with fewer than nev
 * dimensions, the missing pairs are NaN in evals and resid and their evecs
 * slots are not written.  LQ_ERR_ARG for invalid parameters, a zero start
 * vector or a degree with d arccosh((hi + lo) / (hi - lo)) > 600 (T_d would
 * overflow);
 * LQ_NOT_CONVERGED if fewer than nev pairs met tol after max_restarts (the
 * outputs hold the last estimates); with the filter a pair counts as met
 * only if its eigenvalue is at most lo (one above hi, amplified by T_d, is
 * not among the wanted ones).  Synchronizes the stream. */
lq_status lq_eigs(lq_op *op, const lq_eig_params *p, const void *v0, double *evals, double *resid, void *evecs,
                  lq_eig_stats *stats, void *stream);

/* Deflated initial guess for D x = b from eigenpairs (lambda_k, v_k) of
 * A = M^dag M, k < nvec (evals on the host, each finite and > 0; evecs
 * device complex128 [nvec][V/2][4][3], orthonormal, as lq_eigs returns
 * them): the even half x_e = sum_k v_k (v_k^dag M^dag b_hat) / lambda_k is
 * the component of the even-odd solution M^-1 b_hat = A^-1 M^dag b_hat in
 * their span (b_hat = b_e + kappa H_eo A_oo^-1 b_o, the even-odd right-hand
 * side), and the odd half x_o = A_oo^-1 (b_o + kappa H_oe x_e) satisfies the
 * odd rows of D x = b.  b and x0: device complex128 [V][4][3], one
 * right-hand side; x0 is written in full and can be passed to lq_solve with
 * use_x0 = 1, whose residual then lacks those eigenvectors' components.
 * A workspace of 7 packed FP64 fields and 2 even fields stays with the
 * operator (freed with it).  Synchronizes the stream. */
lq_status lq_deflated_guess(lq_op *op, int nvec, const double *evals, const void *evecs, const void *b, void *x0,
                            void *stream);

/* Deflation space of the operator's solves (lq_solver_params.deflate):
 * eigenpairs (lambda_k, v_k) of A = M^dag M, k < nvec <= 1024, evals on the
 * host (finite, > 0), evecs device complex128 [nvec][V/2][4][3] (even
 * sites in checkerboard order, orthonormal, as lq_eigs returns them).  The
 * vectors are copied into device memory of the operator's own (nvec packed
 * FP64 even fields, plus the solves' partial sums), so evecs may be freed
 * after the call; nvec = 0 removes the space (the memory stays until the
 * operator is destroyed).  The space belongs to the current operator:
 * lq_op_set_gauge and lq_op_set_params remove it.  Operators bound to a caller's workspace
 * (lq_op_bind) have no room for it: LQ_ERR_STATE.  The solve stays exact
 * with any vectors (its residual update is an FP64 apply); poor ones only
 * help less.  Synchronizes the stream. */
lq_status lq_op_set_deflation(lq_op *op, int nvec, const double *evals, const void *evecs, void *stream);

/* ------------------------------------------------------------------------
 * Two-level multigrid for D x = b (Sec. 1 cites adaptive multigrid for
 * lattice QCD, Sec. 4 lists multigrid among the solvers; read as
 * adaptive aggregation with a Galerkin coarse operator):
 *   - aggregates: blocks of block[0] x .. x block[3] sites; every coarse
 *     extent L_mu / block_mu must be even and >= 2 (each block_mu >= 2);
 *   - the prolongator P: nvec near-null vectors, each split by chirality
 *     (spins 0, 1 and spins 2, 3) and orthonormalised per aggregate and
 *     chirality (modified Gram-Schmidt in vector order), so P^dag P = 1 and
 *     P commutes with gamma_5; coarse degree of freedom r = chi * nvec + k;
 *   - the coarse operator D_c = P^dag D P, a 9-point stencil of
 *     (2 nvec)^2 complex blocks per coarse site: d = 0 the aggregate
 *     itself, d = 1 + 2 mu the coupling to the aggregate at +mu, d = 2 + 2 mu
 *     to the one at -mu (boundary phases included), stored in FP32;
 *   - the solve: FP64 defect correction around flexible GCR (FP32, restart
 *     gcr_restart) preconditioned by one cycle per iteration: coarse
 *     correction P D_c^-1 P^dag r (BiCGStab on D_c to coarse_tol), then
 *     smooth_steps minimal-residual steps on the fine residual.
 * Near-null vectors: the caller's random start vectors v0, each improved
 * by setup_iters inverse iterations v <- D^-1 v (the operator's own mixed
 * solve to setup_tol, then normalised). */
typedef struct {
    int block[4];         /* aggregate extents (x, y, z, t) */
    int nvec;             /* near-null vectors, 1..32 (coarse dof per site 2 nvec) */
    int setup_iters;      /* inverse iterations per vector (>= 0) */
    double setup_tol;     /* relative residual of those solves, in (0, 1) */
    int smooth_steps;     /* minimal-residual steps of the post-smoother (>= 0) */
    double coarse_tol;    /* relative residual of the coarse solve, in (0, 1) */
    int coarse_max_iter;  /* iteration cap of the coarse solve (>= 1) */
    int gcr_restart;      /* flexible GCR basis length, 1..32 */
} lq_mg_params;

/* block 4^4, nvec 12, setup_iters 3, setup_tol 1e-2, smooth_steps 8,
 * coarse_tol 0.2, coarse_max_iter 200, gcr_restart 16 */
void lq_mg_params_default(lq_mg_params *p);
/* Build the two-level hierarchy for op's current gauge field and
 * parameters (the setup above; it uses the operator's solver).  v0: device
 * complex128 [nvec][V][4][3] start vectors (read only).  The hierarchy keeps
 * a pointer to op (which must outlive it) and its own device memory: nvec
 * FP32 full fields, the coarse operator (9 (2 nvec)^2 complex FP32 per
 * aggregate) and the solver's vectors (2 gcr_restart + 8 FP32 full fields,
 * 3 FP64 full fields).  A new gauge field or new parameters of op need a new
 * hierarchy.  Synchronizes the stream. */
lq_status lq_mg_create(lq_op *op, const lq_mg_params *p, const void *v0, lq_mg **mg, void *stream);
lq_status lq_mg_destroy(lq_mg *mg);
/* D x = b for one right-hand side (device complex128 [V][4][3]; x is
 * written) to the true FP64 residual sp->tol (sp->inner_tol: relative
 * target of each FP32 GCR solve; sp->max_iter caps the GCR iterations,
 * sp->max_outer the FP64 steps; the other fields are not used).  stats:
 * nconv = GCR iterations (one multigrid cycle each), nouter, diff, time.
 * Returns LQ_NOT_CONVERGED if the cap is reached first. */
lq_status lq_mg_solve(lq_mg *mg, const lq_solver_params *sp, void *x, const void *b, lq_solve_stats *stats,
                      void *stream);
/* Parts of the hierarchy, for checks against a reference: the
 * orthonormalised vectors (device complex128 [nvec][V][4][3]); the coarse
 * operator (host complex128 [ncoarse][9][2 nvec][2 nvec], coarse sites
 * lexicographic with x fastest); restriction P^dag f (device complex128
 * fine [V][4][3] -> coarse [ncoarse][2 nvec]), prolongation P c, and
 * y = D_c x on device complex128 coarse vectors.  ncoarse = prod(L / block). */
lq_status lq_mg_vectors(const lq_mg *mg, void *out, void *stream);
lq_status lq_mg_coarse_op(const lq_mg *mg, double *out);
lq_status lq_mg_restrict(lq_mg *mg, const void *fine, void *coarse, void *stream);
lq_status lq_mg_prolong(lq_mg *mg, const void *coarse, void *fine, void *stream);
lq_status lq_mg_coarse_apply(lq_mg *mg, const void *x, void *y, void *stream);

/* ------------------------------------------------------------------------
 * Molecular dynamics of the Monte Carlo gauge-field generation (Sec. 2: the
 * solves of the fermion matrix recur at every step of it), read as hybrid
 * Monte Carlo with the Wilson plaquette gauge action
 *   S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3)
 * and the even-odd pseudofermion action of lq_pf_force (variant 0, the
 * operator's kappa, csw, twist and boundary phases).  Momenta P_mu(x) are traceless
 * anti-Hermitian, H = 1/2 sum tr(P^dag P) + S_g + S_f, and the equations of
 * motion dU/dt = P U, dP/dt = -G (G the su(3) force, -TA(U M) as for
 * lq_pf_force) are integrated with U <- exp(e P) U (FP64).
 * Random numbers are the caller's: P is distributed as exp(-1/2 tr P^dag P)
 * (P = i sum_a xi_a lambda_a / sqrt(2) with Gell-Mann lambda_a and standard
 * normal xi_a), phi = M^dag eta with eta complex Gaussian of density
 * exp(-eta^dag eta) (real and imaginary parts of variance 1/2), and the
 * accept/reject draw compares a uniform r with exp(-dH).
 * ---------------------------------------------------------------------- */
typedef enum { LQ_LEAPFROG = 0, LQ_OMELYAN = 1 } lq_integrator;

typedef struct {
    double beta;          /* gauge coupling (0: no gauge action) */
    double tau;           /* trajectory length */
    int nsteps;           /* integration steps, >= 1 */
    int integrator;       /* lq_integrator: leapfrog (P e/2, U e, P e/2 per step) or the
                             second-order minimum-norm (Omelyan) scheme
                             (P lambda e, U e/2, P (1 - 2 lambda) e, U e/2, P lambda e) */
    double lambda;        /* Omelyan parameter (default 0.1931833275037836) */
    int fermion;          /* 1: with the even-odd pseudofermion action; 0: pure gauge */
    int force_prec;       /* lq_prec of the hopping-term force kernel (LQ_F64 or LQ_F32) */
    int chrono;           /* initial guess of each force solve from the trajectory's previous
                             solutions X: 0 zero, 1 the last X, 2 (default) the linear
                             extrapolation 2 X_last - X_before (solves still run to sp->tol) */
} lq_md_params;

typedef struct {
    double H0, H1, dH;    /* Hamiltonian at the start and the end, dH = H1 - H0 */
    double T0, T1;        /* kinetic terms */
    double Sg0, Sg1;      /* gauge actions */
    double Sf0, Sf1;      /* pseudofermion actions (0 without fermions) */
    int n_force;          /* force evaluations */
    int converged;        /* 1 if every solve reached sp->tol */
    long iters;           /* inner Krylov iterations of all solves */
    double t_ms;          /* wall time */
} lq_md_stats;

/* Defaults: beta 5.6, tau 1, 10 leapfrog steps, lambda 0.1931833275037836,
 * with fermions, FP64 force kernel, chrono 2. */
void lq_md_params_default(lq_md_params *p);

/* Wilson gauge action S (may be NULL) and its su(3) force G (device
 * complex128 [V][4][3][3], may be NULL; G = -TA(U M) with dS = sum Re tr(M dU))
 * on the operator's gauge field.  Synchronizes the stream when S is asked. */
lq_status lq_gauge_force(lq_op *op, double beta, void *G, double *S, void *stream);

/* One molecular-dynamics trajectory from (U, P): U (device complex128 gauge
 * layout) and P (device complex128 [V][4][3][3], traceless anti-Hermitian)
 * are updated in place; the operator is set to U at the start and holds
 * the final U at the end.  phi: device complex128 [V/2][4][3] on the even
 * sites (fermion = 1).  Every force evaluation runs a solve with sp (the
 * solver of lq_pf_force) at the current U, started from the guess chrono
 * selects.  The force and the solution history use a workspace of
 * 4 V 144 + 3 V 96 bytes kept with the operator.  LQ_NOT_CONVERGED if some solve
 * missed sp->tol (stats are filled).  The caller decides acceptance with
 * stats->dH. */
lq_status lq_md_trajectory(lq_op *op, const lq_md_params *mp, const lq_solver_params *sp, void *U, void *P,
                           const void *phi, lq_md_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LQ_H */
