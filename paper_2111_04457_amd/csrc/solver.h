// solver.h -- FP64 defect correction around device-resident Krylov inner
// solvers, shared by the propagator solve and the pseudofermion force.
#pragma once

#include <cstring>
#include <string>
#include <vector>

#include "blas.h"
#include "runtime.h"

// A ragged batch: several lattices (operators of their own volumes and gauge
// fields, nrhs[i] systems each) solved together, every stage of an inner
// iteration one launch over all of them.  Its vectors are ragged fields:
// the even-site slices of every system, lattice by lattice, back to back.
struct lq_batch {
    std::vector<lq_op *> ops;
    std::vector<int> nrhs;
    // layout of the systems (filled by the solve for the current operators)
    std::vector<int> sys0;        // first system of lattice i
    std::vector<long> site0;      // padded sites before lattice i's first slice
    std::vector<long> hop_part0;  // partials of the fused hop reductions before lattice i
    long sites = 0;               // padded sites of all slices
    int nsys = 0;
    int ntiles = 0;               // vector-kernel workgroups over all slices
    lq::Buf tiles;                // lq::Tile[ntiles]
    lq::Buf blas_range;           // int2[nsys]: each system's vector-kernel partials
    lq::Buf hop_range;            // int2[nsys]: each system's fused-hop partials
    lq::Buf ws, sc, partial;      // solver vectors, scalars, partial sums
    double *host_sc = nullptr;    // pinned mirror of the scalars
    size_t host_sc_n = 0;
    std::vector<int> inner_hints;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<lq_op::GraphEntry> graphs;
    std::vector<long> generations;  // of the operators when the graphs were captured
    void clear_graphs()
    {
        for (auto &e : graphs) {
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
            if (e.graph) (void)hipGraphDestroy(e.graph);
        }
        graphs.clear();
    }
    ~lq_batch()
    {
        clear_graphs();
        if (host_sc) (void)hipHostFree(host_sc);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace lq {

// The bits of the twisted mass, for the graph keys (the hop kernels take the
// twist factor as an argument captured into the graph).
inline long twist_key(double t)
{
    long k;
    static_assert(sizeof(k) == sizeof(t), "64-bit long");
    std::memcpy(&k, &t, sizeof(k));
    return k;
}

// Solver context: nsys systems on the solve space (even sites for the
// even-odd Schur system, or the full lattice), workspace and scalars; of one
// operator (op) or of a ragged batch of operators (bt, even-odd only).
struct SolveCtx {
    lq_op *op = nullptr;
    lq_batch *bt = nullptr;
    hipStream_t s = nullptr;
    int nsys = 1;
    bool eo = true;   // even-odd Schur system (else full lattice)
    int sps = 1;      // slices per system of a solve-space vector
    int pin = F64;    // inner storage precision
    int px = F64;     // inner solution precision
    double *sc = nullptr;       // device scalars [nsys][NSC]
    double *hsc = nullptr;      // pinned host mirror
    double *partial = nullptr;  // reduction partials
    char *odd_tmp[3] = {nullptr, nullptr, nullptr};
    long n_hop = 0;
    double hop_bytes = 0;
    // inside an inner-iteration chunk: kernels skip frozen systems and hop
    // applies are counted afterwards from the systems' iteration counters
    bool masked = false;
    bool left = false;   // inner applies use the A_ee^-1-preconditioned Schur operator
    int force_break = 0; // > 0: the first inner BiCGStab solve breaks down at this iteration
    int log = 0;         // progress lines on stderr: 0 none, 1 per solve, 2 per outer step
    bool deflate = false;  // project each outer residual with the operator's deflation space
    // another operator than the fine one (the multigrid coarse operator):
    // apply() calls coarse_apply, which reads coarse; key_extra enters the
    // graph keys (an id of the coarse operator's buffers)
    void (*coarse_apply)(SolveCtx &c, const FieldView &out, const FieldView &in) = nullptr;
    const void *coarse = nullptr;
    long key_extra = 0;
    // FP64 vectors of the solve space
    FieldView x64, r64, y64, t64, aux64;
    // inner vectors
    FieldView ix, ir, ip, iv, is, it, irhat, iw, irin;
    FieldView ex;  // M applied to the inner solution (its precision)

    FieldView space(char *base, int p) const;
    size_t space_bytes(int p) const;
    // groups of systems whose outer-loop decisions are taken together: the
    // whole solve, or each lattice of a batch (so that each lattice's solve
    // is exactly its solve on its own)
    int ngroups() const { return bt ? (int)bt->ops.size() : 1; }
    lq_op *group_op(int g) const { return bt ? bt->ops[g] : op; }
    int group_sys0(int g) const { return bt ? bt->sys0[g] : 0; }
    int group_nsys(int g) const { return bt ? bt->nrhs[g] : nsys; }
    // group g's part of a solve-space vector (an ordinary field of its lattice)
    FieldView group_view(const FieldView &v, int g) const;
    // out = M in on group g alone (its operator's kernels; no mask)
    void apply_group(int g, const FieldView &out, const FieldView &in, bool dag);
    void count_hops(int prec, int n);
    // account 4 hopping applies (two operator applies) per inner iteration
    // the systems performed since the last call
    void count_iterations(std::vector<double> &prev);
    // out = M in (dag: M^dag), in the precision of the views
    void apply(const FieldView &out, const FieldView &in, bool dag);
    void reduce_finish(const FieldView &x, const FieldView &y, int mode, int op_fin);
    // out = M in with <w, out> (mode RED_DOT) or <w, out>, |out|^2
    // (RED_DOT_NORM) reduced and finished with op_fin; fused into the
    // operator's second kernel on the even-odd system
    void apply_reduce_finish(const FieldView &out, const FieldView &in, const FieldView &w, int mode, int op_fin);
    void finish(int K, int op_fin, long n);
    void pull();
    void push();
    // Run `chunk` iterations of body(); with graphs enabled the chunk is
    // captured once into a hipGraph (keyed by kind, chunk and every buffer
    // and setting the kernels read) and replayed.
    template <typename Body> void run_chunk(int kind, int chunk, Body body);
};

// Lengths of the inner-iteration chunks of one inner solve.  The host reads
// the scalars back after each chunk; a system that converges inside a chunk
// is masked for the rest of it, so the lengths change only how many masked
// (nearly empty) iterations are launched, never a result.  The first chunk
// is the iteration count of the same-numbered inner solve of the operator's
// previous solve (the first inner solve starts from b, the later ones from
// residuals an inner solve already reduced), else of the previous inner
// solve of this one; then one short chunk, then check_every.
struct ChunkPlan {
    int hint = 0;   // iterations the previous inner solve needed (0: none yet)
    int every = 10;
    int done = 0;   // iterations launched in this inner solve
    int extra = 0;  // chunks launched past the hint
    void start(int check_every)
    {
        every = check_every < 1 ? 1 : check_every;
        done = extra = 0;
    }
    int next(int budget_left)
    {
        int c;
        if (hint > done) c = hint - done < every ? hint - done : every;
        else c = (extra++ == 0 && every > 2) ? 2 : every;
        if (c > budget_left) c = budget_left;
        done += c;
        return c < 1 ? 1 : c;
    }
    // after the inner solve: the most iterations a live system made
    void learn(const SolveCtx &c);
};

template <typename Body> void SolveCtx::run_chunk(int kind, int chunk, Body body)
{
    if (!(bt ? bt->ops[0]->use_graphs : op->use_graphs)) {
        for (int k = 0; k < chunk; ++k) body();
        return;
    }
    // the graph replays the chunk with the masking state it was captured with
    const long masked_key = masked ? 1 : 0;
    std::vector<long> key = {kind, chunk, nsys, eo ? 1 : 0, pin, px, (long)partial, (long)sc, (long)(void *)s,
                             masked_key, left ? 1L : 0L, key_extra};
    if (bt) {
        // every pointer and launch setting the batched kernels read
        key.push_back((long)bt->ws.ptr);
        key.push_back((long)bt->ws.bytes);
        key.push_back((long)bt->tiles.ptr);
        for (const lq_op *o : bt->ops) key.push_back(o->generation);
    } else {
        const long k2[] = {(long)op->solver_ws.ptr, (long)op->solver_ws.bytes,
                           (long)op->hop_block[0], (long)op->hop_block[1], (long)op->hop_block[2],
                           (long)op->xcd_remap[0], (long)op->xcd_remap[1], (long)op->xcd_remap[2],
                           (long)op->rhs_per_thread[0], (long)op->rhs_per_thread[1], (long)op->rhs_per_thread[2],
                           (long)op->halo[2], twist_key(op->prm.twist)};
        key.insert(key.end(), k2, k2 + sizeof(k2) / sizeof(k2[0]));
    }
    std::vector<lq_op::GraphEntry> &graphs = bt ? bt->graphs : op->graphs;
    lq_op::GraphEntry *e = nullptr;
    for (auto &g : graphs)
        if (g.key == key) e = &g;
    if (!e) {
        lq_op::GraphEntry ne;
        ne.key = key;
        const long n0 = n_hop;
        const double b0 = hop_bytes;
        LQ_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            for (int k = 0; k < chunk; ++k) body();
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        LQ_HIP(hipStreamEndCapture(s, &ne.graph));
        LQ_HIP(hipGraphInstantiate(&ne.exec, ne.graph, nullptr, nullptr, 0));
        ne.n_hop = n_hop - n0;
        ne.hop_bytes = hop_bytes - b0;
        n_hop = n0;
        hop_bytes = b0;
        graphs.push_back(ne);
        e = &graphs.back();
    }
    LQ_HIP(hipGraphLaunch(e->exec, s));
    n_hop += e->n_hop;
    hop_bytes += e->hop_bytes;
}

// Allocate the workspace of a solve of nsys systems with inner precision
// `inner` on the even-odd (eo) or full-lattice space.
void make_ctx(SolveCtx &c, lq_op *op, int nsys, bool eo, int inner, hipStream_t s);
// Point the solver's vectors of c (space, precisions set) into base; odd:
// bytes of each odd temporary.
void carve_vectors(SolveCtx &c, char *base, size_t odd);

struct OuterStats {
    std::vector<int> iters, outer, restarts;
    std::vector<double> r2;  // |rhs - A x|^2 at the returned x (FP64)
};

// Solve A x = rhs on the solve space to |rhs - A x|^2 <= target2[i] for
// each system, A = M (normal = false; BiCGStab on M or CG on M^dag M) or
// A = M^dag M (normal = true; CG).  x (c.x64) holds the initial guess;
// x_zero says it is zero (the first residual is then rhs, no apply).
OuterStats defect_correction(SolveCtx &c, const lq_solver_params &sp, bool normal, const FieldView &rhs,
                             const std::vector<double> &target2, bool x_zero);

// Inner Krylov pieces: initialisation from e = 0 and one iteration,
// launched on c.s (used by the single solve and by the batched solve).
void bicg_init(SolveCtx &c);
void bicg_iter(SolveCtx &c);
void cg_init(SolveCtx &c, bool normal_rhs);
void cg_iter(SolveCtx &c);
bool all_frozen(const SolveCtx &c);
// Reliable-update restarts of the inner solvers: the residual replaced by
// the new source c.irin, the search directions kept (SC_REINIT = 0).
void bicg_restart(SolveCtx &c);
void cg_restart(SolveCtx &c, bool normal_rhs);
// One inner BiCGStab solve from e = 0 on c's operator with source c.irin
// (SC_TARGET2 set relative, SC_ODONE clear): chunks of check_every
// iterations after a first one of hint (updated to the iterations needed);
// returns the iterations launched.
int bicgstab_solve(SolveCtx &c, int max_iter, int check_every, int &hint);

// Deflation of the outer residual r (c.r64) with the operator's deflation
// space: x += e, r -= A e for e = sum_k v_k v_k^dag y / lambda_k, y = M^dag r
// (A = M) or r (normal: A = M^dag M); then FIN_NORM of the new r.  Uses
// c.y64 and c.t64.  One operator, even-odd space.
void deflate_residual(SolveCtx &c, bool normal);

// Solve D x = b for nsys systems on full packed FP64 fields ([rhs][parity])
// with the operator's mixed-precision solver (stats per system).
lq_status solve_packed(lq_op *op, const lq_solver_params &sp, int nsys, char *x64, const char *b64, bool use_x0,
                       lq_solve_stats *stats, hipStream_t s);

// Host-side validation of solver parameters; why holds the reason.
bool valid_solver_params(const lq_solver_params *sp, std::string &why);

// |v|^2 per system of a field with sps slices per system.
std::vector<double> norms2(SolveCtx &c, const FieldView &v, int sps);

// The batched Schur operator over every lattice of c.bt (two launches of the
// batched hopping kernel), with the fused reductions of hop() (red, w).
void batch_schur(SolveCtx &c, int prec, const FieldView &out, const FieldView &in, const FieldView &odd, bool dag,
                 bool left, int red, const FieldView *w);


// The pseudofermion force of lq_pf_force with an initial guess X0 for the
// even-odd solve (device complex128 [V/2][4][3], or null for zero).
lq_status pf_force_guess(lq_op *op, const lq_solver_params *sp, int variant, lq_prec force_prec, const void *phi,
                         void *dSdU, void *G, void *X_out, double *S, lq_solve_stats *stats, void *stream,
                         const void *X0);

}  // namespace lq
