// runtime.hip -- operator applies on packed fields.
#include "runtime.h"

#include <algorithm>
#include <cstdlib>

#include "blas.h"

namespace lq {

// layout of the solver scalars read as a freeze mask by the hop kernels
constexpr int MASK_STRIDE = NSC, MASK_DONE = SC_DONE, MASK_BREAK = SC_BREAK;

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *get_error() { return g_last_error.c_str(); }

void Buf::release()
{
    if (ptr && !borrowed) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    borrowed = false;
}

void Buf::borrow(char *p, size_t n)
{
    release();
    ptr = p;
    bytes = n;
    borrowed = true;
}

void Buf::ensure(size_t n)
{
    if (n <= bytes && (ptr || borrowed)) return;
    if (borrowed)
        throw Failure{LQ_ERR_NOMEM, "the bound workspace is too small for this call (a region of " +
                                        std::to_string(bytes) + " bytes, " + std::to_string(n) +
                                        " needed): bind one of lq_op_workspace_bytes bytes for its nrhs"};
    release();
    if (n == 0) n = 256;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Failure{LQ_ERR_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed: " + hipGetErrorString(e)};
    }
    ptr = static_cast<char *>(p);
    bytes = n;
}

bool kind_is_full(lq_kind k) { return k == LQ_D || k == LQ_DDAG || k == LQ_DDAGD; }

int log_level(const lq_op *op)
{
    static const int env = [] {
        const char *v = std::getenv("LQ_LOG_LEVEL");
        return v ? std::atoi(v) : 0;
    }();
    return std::max(env, op ? op->log_level : 0);
}

void twist_factor(const lq_op *op, bool inv, bool dag, double &re, double &im)
{
    // A = 1 + i tau gamma_5 on spins 0, 1: 1 + i tau; A^-1: (1 - i tau) / (1 + tau^2);
    // the dagger conjugates
    const double t = op->prm.twist;
    if (inv) {
        re = 1.0 / (1.0 + t * t);
        im = -t / (1.0 + t * t);
    } else {
        re = 1.0;
        im = t;
    }
    if (dag) im = -im;
}

HopArgs hop_args(lq_op *op, int prec, const FieldView &out, const FieldView &in, int p_out, int clov_mode, bool inv,
                 bool dag, const FieldView *y, double coef, const FieldView *w)
{
    const Geom &g = op->g;
    HopArgs a{};
    a.g = g;
    a.p_out = p_out;
    a.nrhs = in.nrhs;
    a.in = in.base;
    a.in_n = in.n;
    a.in_rs = in.rs;
    a.out = out.base;
    a.out_n = out.n;
    a.out_rs = out.rs;
    if (y) {
        a.y = y->base;
        a.y_n = y->n;
        a.y_rs = y->rs;
    }
    if (w) {
        a.w = w->base;
        a.w_n = w->n;
        a.w_rs = w->rs;
    }
    a.links = op->hop_links(prec);
    if (clov_mode && op->has_clover)
        a.clov = (inv ? op->clovinv[prec].ptr : op->clov[prec].ptr) + (long)p_out * clover_bytes(prec, g.vh);
    else if (clov_mode && op->has_twist)
        twist_factor(op, inv, dag, a.tw_re, a.tw_im);
    a.coef = coef;
    return a;
}

void hop(lq_op *op, int prec, const FieldView &out, const FieldView &in, int p_out, bool dag, int clov_mode,
         bool inv, const FieldView *y, double coef, int red, const FieldView *w, hipStream_t s)
{
    if (out.tiles || in.tiles) throw Failure{LQ_ERR_STATE, "hop: a ragged field needs the batched hopping kernel"};
    const Geom &g = op->g;
    HopArgs a = hop_args(op, prec, out, in, p_out, clov_mode, inv, dag, y, coef, w);
    if (clov_mode && !op->has_clover && !op->has_twist) clov_mode = 0;
    if (clov_mode && op->has_twist) clov_mode |= kTwist;
    if (op->hop_mask) set_hop_mask(a, op->hop_mask);
    if (red) {
        // one partial per 64-site wavefront and right-hand side, K <= 3
        op->partial.ensure((size_t)((g.vh + 63) / 64) * in.nrhs * 3 * sizeof(double));
        a.partial = reinterpret_cast<double *>(op->partial.ptr);
    }
    // neighbour spinors staged in LDS (binary16, one right-hand side)
    HaloTile tile;
    if (op->halo[prec] && prec == F16 && in.nrhs == 1 && !(clov_mode & kTwist) && halo_tile(g, tile)) {
        LQ_HIP(launch_hop_halo(a, tile, prec, op->nl(prec), dag, clov_mode, y != nullptr, red, s));
        return;
    }
    // right-hand sides per thread (2, no reductions), or 4 per workgroup
    // sharing the links in LDS (at least 4 right-hand sides)
    int nr = 1;
    if (in.nrhs > 1) {
        const int want = eff_nr(op, prec, in.nrhs);
        if (want == 2 && red == 0) nr = 2;
        else if (want == 4 && in.nrhs >= 4) nr = 4;
    }
    const int remap = eff_remap(op, prec, in.nrhs);
    a.xcd_remap = remap != 0 ? 1 : 0;
    const int block = op->hop_block[prec];
    if (remap == 2) {
        const long slice = (long)g.L[0] * g.L[1] * g.L[2] / 2;  // sites of one parity per time slice
        const int sb = nr == 4 ? 64 : block;                     // sites per tile
        if (slice % sb == 0) {
            a.slice_tiles = (int)(slice / sb);
            a.tgroup = std::max(1, g.L[3] / 8);  // one group of slices per XCD
        }
    }
    LQ_HIP(launch_hop(a, prec, op->nl(prec), dag, clov_mode, y != nullptr, red, nr, block, s));
}

int eff_remap(const lq_op *op, int prec, int nrhs)
{
    const int v = op->xcd_remap[prec];
    return v >= 0 ? v : (nrhs > 1 ? 2 : 0);
}

int eff_nr(const lq_op *op, int prec, int nrhs)
{
    // measured at 24^3 x 48 and 32^3 x 64: four per workgroup from four
    // right-hand sides on (every precision), two per thread for two or three
    // in FP16 (its dot-product arithmetic leaves the registers for them)
    const int v = op->rhs_per_thread[prec];
    if (v > 0) return v;
    if (nrhs >= 4) return 4;
    return prec == F16 && nrhs >= 2 ? 2 : 1;
}

void set_hop_mask(HopArgs &a, const double *sc)
{
    a.mask = sc;
    a.mask_stride = MASK_STRIDE;
    a.mask_off0 = MASK_DONE;
    a.mask_off1 = MASK_BREAK;
}

void clover_apply(lq_op *op, int prec, int p, bool inv, const FieldView &out, const FieldView &in, hipStream_t s)
{
    if (!op->has_clover && op->has_twist) {
        double re, im;
        twist_factor(op, inv, false, re, im);
        LQ_HIP(launch_twist_apply(op->g, re, im, out, in, s));
        return;
    }
    if (!op->has_clover) {
        if (out.base != in.base)
            for (int r = 0; r < in.nrhs; ++r)
                LQ_HIP(hipMemcpyAsync(out.base + r * out.rs, in.base + r * in.rs, fb(prec, op->g),
                                      hipMemcpyDeviceToDevice, s));
        return;
    }
    const char *c = (inv ? op->clovinv[prec].ptr : op->clov[prec].ptr) + (long)p * clover_bytes(prec, op->g.vh);
    LQ_HIP(launch_clover_apply(op->g, c, out, in, s));
}

// Schur operator M = A_ee - kappa^2 H_eo A_oo^-1 H_oe (dag: M^dag) on packed
// even fields; t is an odd scratch field.
void schur(lq_op *op, int prec, const FieldView &out, const FieldView &in, const FieldView &t, bool dag,
           hipStream_t s, int red, const FieldView *w)
{
    const double k = op->prm.kappa;
    hop(op, prec, t, in, 1, dag, 2, true, nullptr, 1.0, 0, nullptr, s);
    hop(op, prec, out, t, 0, dag, 1, false, &in, -k * k, red, w, s);
}

// The A_ee^-1-preconditioned Schur operator A_ee^-1 M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe
// (needs ensure_even_inverse first).
void schur_left(lq_op *op, int prec, const FieldView &out, const FieldView &in, const FieldView &t, hipStream_t s,
                int red, const FieldView *w)
{
    const double k = op->prm.kappa;
    hop(op, prec, t, in, 1, false, 2, true, nullptr, 1.0, 0, nullptr, s);
    hop(op, prec, out, t, 0, false, 3, true, &in, -k * k, red, w, s);
}

// A_ee^-1 (the even blocks; the odd ones are inverted with the clover
// build), in FP64 and converted to every precision, on first use.
void ensure_even_inverse(lq_op *op, hipStream_t s)
{
    if (!op->has_clover || op->even_inverted) return;
    const Geom &g = op->g;
    LQ_HIP(hipMemsetAsync(op->flag.ptr, 0, sizeof(int), s));
    LQ_HIP(launch_clover_invert(g, 0, op->clov[F64].ptr, op->clovinv[F64].ptr, reinterpret_cast<int *>(op->flag.ptr),
                                s));
    for (int p = F32; p <= F16; ++p)
        LQ_HIP(launch_convert_clover(g, op->clovinv[F64].ptr, p, op->clovinv[p].ptr, s, 0, 1));
    int flag = 0;
    LQ_HIP(hipMemcpyAsync(&flag, op->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
    if (flag) throw Failure{LQ_ERR_SINGULAR, "a clover block A_ee = 1 + F on an even site is singular"};
    op->even_inverted = true;
}

// Full-lattice D (or D^dag): out_p = A_pp in_p - kappa H_{p,1-p} in_{1-p}.
void dirac_full(lq_op *op, int prec, char *out, const char *in, int nrhs, bool dag, hipStream_t s)
{
    const Geom &g = op->g;
    for (int p = 0; p < 2; ++p) {
        const FieldView o = full_parity_view(out, prec, g, nrhs, p);
        const FieldView x_in = full_parity_view(const_cast<char *>(in), prec, g, nrhs, 1 - p);
        const FieldView y = full_parity_view(const_cast<char *>(in), prec, g, nrhs, p);
        hop(op, prec, o, x_in, p, dag, 1, false, &y, -op->prm.kappa, 0, nullptr, s);
    }
}

void apply_temp_bytes(lq_kind kind, int prec, const Geom &g, int nrhs, size_t &t0, size_t &t1)
{
    t0 = t1 = 0;
    switch (kind) {
    case LQ_DDAGD: t0 = 2 * (size_t)fb(prec, g) * nrhs; break;
    case LQ_SCHUR:
    case LQ_SCHUR_DAG:
    case LQ_SCHUR_LEFT: t0 = (size_t)fb(prec, g) * nrhs; break;
    case LQ_SCHUR_NORMAL: t0 = t1 = (size_t)fb(prec, g) * nrhs; break;
    default: break;
    }
}

void apply_packed(lq_op *op, lq_kind kind, int prec, char *out, const char *in, int nrhs, hipStream_t s, char *t0,
                  char *t1)
{
    const Geom &g = op->g;
    const FieldView o = parity_view(out, prec, g, nrhs);
    const FieldView i = parity_view(const_cast<char *>(in), prec, g, nrhs);
    size_t b0, b1;
    apply_temp_bytes(kind, prec, g, nrhs, b0, b1);
    if (b0 && !t0) {
        op->tmp[0].ensure(b0);
        t0 = op->tmp[0].ptr;
    }
    if (b1 && !t1) {
        op->tmp[1].ensure(b1);
        t1 = op->tmp[1].ptr;
    }
    switch (kind) {
    case LQ_D: dirac_full(op, prec, out, in, nrhs, false, s); break;
    case LQ_DDAG: dirac_full(op, prec, out, in, nrhs, true, s); break;
    case LQ_DDAGD: {
        dirac_full(op, prec, t0, in, nrhs, false, s);
        dirac_full(op, prec, out, t0, nrhs, true, s);
        break;
    }
    case LQ_SCHUR:
    case LQ_SCHUR_DAG: {
        schur(op, prec, o, i, parity_view(t0, prec, g, nrhs), kind == LQ_SCHUR_DAG, s);
        break;
    }
    case LQ_SCHUR_NORMAL: {
        const FieldView t = parity_view(t0, prec, g, nrhs);
        const FieldView m = parity_view(t1, prec, g, nrhs);
        schur(op, prec, m, i, t, false, s);
        schur(op, prec, o, m, t, true, s);
        break;
    }
    case LQ_HOP_EO: hop(op, prec, o, i, 0, false, 0, false, nullptr, 1.0, 0, nullptr, s); break;
    case LQ_HOP_OE: hop(op, prec, o, i, 1, false, 0, false, nullptr, 1.0, 0, nullptr, s); break;
    case LQ_HOP_EO_DAG: hop(op, prec, o, i, 0, true, 0, false, nullptr, 1.0, 0, nullptr, s); break;
    case LQ_HOP_OE_DAG: hop(op, prec, o, i, 1, true, 0, false, nullptr, 1.0, 0, nullptr, s); break;
    case LQ_CLOVER_E: clover_apply(op, prec, 0, false, o, i, s); break;
    case LQ_CLOVER_O: clover_apply(op, prec, 1, false, o, i, s); break;
    case LQ_CLOVER_INV_O: clover_apply(op, prec, 1, true, o, i, s); break;
    case LQ_SCHUR_LEFT: {
        ensure_even_inverse(op, s);
        schur_left(op, prec, o, i, parity_view(t0, prec, g, nrhs), s);
        break;
    }
    default: throw Failure{LQ_ERR_ARG, "unknown operator kind"};
    }
}

}  // namespace lq
