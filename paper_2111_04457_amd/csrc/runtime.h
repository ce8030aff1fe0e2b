// runtime.h -- host-side runtime of the library: device buffers, the
// operator object (packed links and clover in every precision), operator
// applies on packed fields, and error reporting for the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lq.h"
#include "dslash.h"
#include "fields.h"

namespace lq {

// Thread-local message of the last failure, returned by lq_last_error().
void set_error(const std::string &msg);
const char *get_error();

// An error carried out of the runtime to the ABI, with its status code.
struct Failure {
    lq_status code;
    std::string msg;
};

#define LQ_HIP(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            throw ::lq::Failure{LQ_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)};    \
    } while (0)

// A device buffer: allocated by the library (owned), or a region of a
// workspace the caller bound to the operator (borrowed; never reallocated).
struct Buf {
    char *ptr = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    Buf() = default;
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    ~Buf() { release(); }
    void release();
    // make sure at least n bytes are available (contents are not kept); a
    // borrowed region that is too small is an error, not a reallocation
    void ensure(size_t n);
    // use [p, p + n) of a caller's allocation
    void borrow(char *p, size_t n);
    size_t owned() const { return borrowed ? 0 : bytes; }
};

}  // namespace lq

struct lq_op {
    lq_op_params prm;
    lq::Geom g;
    int device = 0;
    bool gauge_set = false;
    bool has_clover = false;
    bool has_twist = false;              // twisted-mass Wilson operator (prm.twist != 0, no clover)
    bool even_inverted = false;          // A_ee^-1 computed for the current gauge field
    int hop_block[3] = {64, 64, 64};     // workgroup size of the hop kernel per precision
    // workgroup order of the hop kernel per precision: 0 plain, 1 XCD-aware,
    // 2 XCD-aware and time slices interleaved; -1 automatic (eff_remap)
    int xcd_remap[3] = {-1, -1, -1};
    int tune_form = 0;                   // operator form lq_tune times: 0 M, 1 A_ee^-1 M
    int break_at = 0;                    // > 0: the next solve's first inner BiCGStab breaks down here
    int log_level = 0;                   // progress lines of solves on stderr (also $LQ_LOG_LEVEL)
    int rhs_per_thread[3] = {0, 0, 0};   // right-hand sides per thread of the hop kernel (nrhs > 1); 0 automatic
    int halo[3] = {0, 0, 0};             // 1: neighbour spinors staged in LDS (binary16, one rhs, if a tile fits)
    std::vector<int> inner_hints;        // iterations the k-th inner solve of the last solve needed
                                         // (first chunk length of the next solve's k-th)
    lq::Buf links[3];                    // packed links per precision ([parity][mu]); FP64 always 18 reals
    lq::Buf links64r;                    // FP64 links with 12 reals (hop kernels) when link_recon == 12
    lq::Buf clov[3];                     // A = 1 + F per precision ([parity])
    lq::Buf clovinv[3];                  // A^-1 per precision ([parity])
    lq::Buf flag;                        // device int: singular clover block
    // scratch fields: 0, 1 temporaries of composite applies; 2, 3 packed
    // input / output of an apply; 4, 5 packed b and x of a solve; 6, 7
    // staging of host inputs and outputs
    lq::Buf tmp[8];
    lq::Buf force_ws;                    // clover-force insertions ([parity][plane], FP64)
    lq::Buf defl_ws[3];                  // deflated guess: packed fields, even fields, partial sums
    lq::Buf defl_vecs;                   // deflation space: packed FP64 eigenvectors, then 1 / lambda
    lq::Buf defl_part;                   // deflation: partial sums and coefficients of the projection
    int defl_n = 0;                      // vectors of the deflation space (0: none)
    lq::Buf md_G;                        // molecular dynamics: the force on every link
    lq::Buf md_partial;                  // molecular dynamics: per-wavefront partial sums
    lq::Buf md_X[3];                     // molecular dynamics: previous solutions and the next guess
    lq::Buf eig_ws[8];                   // eigensolver: Krylov basis, Ritz vectors, work vector, packed
                                         // fields, partial sums, projections, coefficients, rotation
    double *eig_host = nullptr;          // eigensolver: pinned host scalars
    lq::Buf partial;                     // reduction partial sums
    lq::Buf solver_ws;                   // solver work vectors
    lq::Buf solver_sc;                   // solver scalars (device)
    double *host_sc = nullptr;           // pinned host mirror of the solver scalars
    size_t host_sc_n = 0;
    int bound_nrhs = 0;                  // > 0: device memory is the caller's bound workspace, laid
                                         // out for this many right-hand sides
    int use_graphs = 1;                  // capture inner-iteration chunks in hipGraphs
    const double *hop_mask = nullptr;    // per-system freeze flags for hop kernels (set by the solvers)
    hipStream_t stream = nullptr;        // internal stream of solves (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // captured inner-iteration chunks, keyed by everything the kernels read
    struct GraphEntry {
        std::vector<long> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        long n_hop = 0;
        double hop_bytes = 0;
    };
    std::vector<GraphEntry> graphs;
    long generation = 0;                 // bumped whenever captured graphs become stale
    void clear_graphs()
    {
        ++generation;
        for (auto &e : graphs) {
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
            if (e.graph) (void)hipGraphDestroy(e.graph);
        }
        graphs.clear();
    }
    ~lq_op()
    {
        clear_graphs();
        if (host_sc) (void)hipHostFree(host_sc);
        if (eig_host) (void)hipHostFree(eig_host);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (stream) (void)hipStreamDestroy(stream);
    }
    // device bytes of the work buffers allocated on demand (temporaries,
    // reduction partials, solver, force, eigensolver and MD workspaces)
    size_t work_bytes() const
    {
        size_t n = force_ws.bytes + md_G.bytes + md_partial.bytes + partial.bytes + solver_ws.bytes + solver_sc.bytes +
                   defl_vecs.bytes + defl_part.bytes;
        for (const auto &b : tmp) n += b.bytes;
        for (const auto &b : defl_ws) n += b.bytes;
        for (const auto &b : md_X) n += b.bytes;
        for (const auto &b : eig_ws) n += b.bytes;
        return n;
    }
    // device bytes the library allocated itself for this operator (not
    // counting regions of a bound workspace)
    size_t owned_bytes() const
    {
        size_t n = links64r.owned() + flag.owned() + force_ws.owned() + md_G.owned() + md_partial.owned() +
                   partial.owned() + solver_ws.owned() + solver_sc.owned() + defl_vecs.owned() + defl_part.owned();
        for (int p = 0; p < 3; ++p) n += links[p].owned() + clov[p].owned() + clovinv[p].owned();
        for (const auto &b : tmp) n += b.owned();
        for (const auto &b : defl_ws) n += b.owned();
        for (const auto &b : md_X) n += b.owned();
        for (const auto &b : eig_ws) n += b.owned();
        return n;
    }
    // link format of the hop kernels (the clover build and the force use the
    // 18-real FP64 links)
    int nl(int) const { return prm.link_recon; }
    const char *hop_links(int prec) const
    {
        return (prec == lq::F64 && prm.link_recon == 12) ? links64r.ptr : links[prec].ptr;
    }
};

struct lq_field {
    lq_op *op;
    int prec;
    int nrhs;
    lq::Buf data;
    lq::FieldView view() const
    {
        return lq::FieldView{data.ptr, prec, (long)op->g.vh, lq::spinor_field_bytes(prec, op->g.vh), nrhs};
    }
};

namespace lq {

inline long fb(int prec, const Geom &g) { return spinor_field_bytes(prec, g.vh); }

// A parity field view on buffer memory (nrhs slices, contiguous).
inline FieldView parity_view(char *base, int prec, const Geom &g, int nrhs)
{
    return FieldView{base, prec, (long)g.vh, fb(prec, g), nrhs};
}
// Parity p of a full packed field laid out [rhs][parity][planes].
inline FieldView full_parity_view(char *base, int prec, const Geom &g, int nrhs, int p)
{
    return FieldView{base + p * fb(prec, g), prec, (long)g.vh, 2 * fb(prec, g), nrhs};
}

// Arguments of the hopping kernel for out = epilogue(coef * H_{p_out,1-p_out} in)
// on op's links and clover blocks (default launch shape, no mask, no
// reduction partials).
HopArgs hop_args(lq_op *op, int prec, const FieldView &out, const FieldView &in, int p_out, int clov_mode, bool inv,
                 bool dag, const FieldView *y, double coef, const FieldView *w);
// The twisted-mass factor on spins 0, 1 of A = 1 + i tau gamma_5 (inv: of A^-1;
// dag: conjugated); spins 2, 3 take its conjugate.
void twist_factor(const lq_op *op, bool inv, bool dag, double &re, double &im);
// Freeze mask of the hopping kernel: the solver scalars sc of its right-hand sides.
void set_hop_mask(HopArgs &a, const double *sc);

// Hopping term on packed fields: out = epilogue(coef * H_{p_out,1-p_out} in).
// clov_mode: 0 none, 1 clover on y, 2 clover on the result; inv selects A^-1.
// red: 0 none, 2 per-rhs <w, out>, 3 <w, out> and |out|^2, as per-wavefront
// partials into op->partial (see launch_hop).
void hop(lq_op *op, int prec, const FieldView &out, const FieldView &in, int p_out, bool dag, int clov_mode,
         bool inv, const FieldView *y, double coef, int red, const FieldView *w, hipStream_t s);

// Apply kind on packed fields of precision prec.  Full kinds take full
// packed fields ([rhs][parity][planes]); the others parity fields.
// t0, t1: temporaries of apply_temp_bytes(kind, ...) bytes each, or null
// for the operator's own (allocated on first use).
void apply_packed(lq_op *op, lq_kind kind, int prec, char *out, const char *in, int nrhs, hipStream_t s,
                  char *t0 = nullptr, char *t1 = nullptr);
// Bytes of each of the temporaries t0 / t1 apply_packed needs for kind
// (0 if that temporary is not used).
void apply_temp_bytes(lq_kind kind, int prec, const Geom &g, int nrhs, size_t &t0, size_t &t1);

// Clover of parity p (inverse if inv) applied site-locally.
void clover_apply(lq_op *op, int prec, int p, bool inv, const FieldView &out, const FieldView &in, hipStream_t s);

bool kind_is_full(lq_kind k);

// The launch settings in effect for nrhs right-hand sides of precision prec:
// the option's value, or, automatic (-1 / 0), plain order for one right-hand
// side and XCD-aware order with the time slices interleaved for several;
// four right-hand sides per workgroup with at least four,
// two per thread in FP16 with two or three, else one per thread (the
// measured best untuned shapes on 24^3 x 48 and 32^3 x 64).
int eff_remap(const lq_op *op, int prec, int nrhs);
int eff_nr(const lq_op *op, int prec, int nrhs);

// Progress output level of solves: the larger of $LQ_LOG_LEVEL (read once)
// and the operator's "log_level" option.
int log_level(const lq_op *op);

// Geometry of the lattice of p (dims, parity split, boundary phases).
Geom make_geom(const lq_op_params &p);

// The regions of an operator's device memory for calls of up to nrhs
// right-hand sides: packed links and clover blocks (per gauge field) and the
// work buffers of applies and solves, each starting on a 256-byte boundary.
struct WorkspaceLayout {
    enum Region {
        LINKS64, LINKS32, LINKS16, LINKS64R, CLOV64, CLOV32, CLOV16, CLOVINV64, CLOVINV32, CLOVINV16, FLAG,
        TMP0, TMP1, TMP2, TMP3, TMP4, TMP5, TMP6, TMP7, PARTIAL, SOLVER_SC, SOLVER_WS, NREGION
    };
    size_t off[NREGION] = {};
    size_t size[NREGION] = {};
    size_t total = 0;
};
WorkspaceLayout workspace_layout(const lq_op_params &p, int nrhs);

// Bytes of the solver workspace of nsys systems (solve space even-odd or full
// lattice, inner storage precision inner).
size_t solver_ws_bytes(const Geom &g, int nsys, bool eo, int inner);

// Schur operator M (or M^dag) on packed even fields; t: odd scratch field.
// red / w: reduction fused into the second kernel (as for hop).
void schur(lq_op *op, int prec, const FieldView &out, const FieldView &in, const FieldView &t, bool dag,
           hipStream_t s, int red = 0, const FieldView *w = nullptr);
// The A_ee^-1-preconditioned Schur operator 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe
// (ensure_even_inverse first; no dagger form).
void schur_left(lq_op *op, int prec, const FieldView &out, const FieldView &in, const FieldView &t, hipStream_t s,
                int red = 0, const FieldView *w = nullptr);
// Invert the even clover blocks (once per gauge field); LQ_ERR_SINGULAR if one is singular.
void ensure_even_inverse(lq_op *op, hipStream_t s);
// Full-lattice D (or D^dag) on full packed fields of nrhs systems.
void dirac_full(lq_op *op, int prec, char *out, const char *in, int nrhs, bool dag, hipStream_t s);

}  // namespace lq
