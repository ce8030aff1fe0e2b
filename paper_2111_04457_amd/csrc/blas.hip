// blas.hip -- vector kernels and device-side scalar recurrences of the
// Krylov solvers.  Sums are accumulated in FP64 whatever the storage
// precision; every reduction is summed in a fixed order.
#include <cmath>

#include "blas.h"

namespace lq {

constexpr int BT = 256;  // threads per workgroup of the vector kernels

int blas_blocks(long n) { return (int)((n + BT - 1) / BT); }

template <typename R> __device__ __forceinline__ cx<R> scal(const double *sc, int slot)
{
    return cx<R>{(R)sc[slot], (R)sc[slot + 1]};
}

__device__ __forceinline__ bool frozen(const double *sc) { return sc[SC_DONE] != 0.0 || sc[SC_BREAK] != 0.0; }

// The site of this thread: slice, site index i, the slice's length n, and
// the index of this workgroup's partial sum (one per workgroup, slice by
// slice).  A uniform field's grid is (sites / BT, slices); a ragged one's
// (tiles).
struct Loc {
    long i;
    int slice;
    long n;
    long site_off;  // ragged: padded sites before the slice; uniform: -1
    long part;
};

__device__ __forceinline__ Loc locate(const FieldView &x)
{
    Loc l;
    if (x.tiles) {
        const Tile t = x.tiles[blockIdx.x];
        l.i = (long)t.blk * BT + threadIdx.x;
        l.slice = t.slice;
        l.n = t.n;
        l.site_off = t.site_off;
        l.part = blockIdx.x;
    } else {
        l.i = (long)blockIdx.x * BT + threadIdx.x;
        l.slice = blockIdx.y;
        l.n = x.n;
        l.site_off = -1;
        l.part = (long)blockIdx.y * gridDim.x + blockIdx.x;
    }
    return l;
}

// Base of this thread's slice in field v (of v's own precision).
__device__ __forceinline__ char *at(const FieldView &v, const Loc &l)
{
    return l.site_off >= 0 ? v.base + l.site_off * (spinor_field_bytes(v.prec, SB) / SB) : v.base + l.slice * v.rs;
}

// ------------------------------------------------------------ reductions --

template <int P, int MODE>
__global__ __launch_bounds__(BT) void reduce_kernel(FieldView x, FieldView y, double *partial, const double *mask,
                                                   int sps)
{
    using R = typename PT<P>::R;
    const Loc L = locate(x);
    const long i = L.i;
    const int slice = L.slice;
    double a = 0, b = 0, c = 0;
    const bool live = !mask || !frozen(mask + (slice / sps) * NSC);
    if (i < L.n && live) {
        const Spinor<R> xv = load_spinor<P>(at(x, L), i, L.n);
        if constexpr (MODE == RED_NORM) {
#pragma unroll
            for (int k = 0; k < 12; ++k) a += (double)norm2(xv.c[k]);
        } else {
            const Spinor<R> yv = load_spinor<P>(at(y, L), i, L.n);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cx<R> t = cmulc(xv.c[k], yv.c[k]);
                a += (double)t.re;
                b += (double)t.im;
                if constexpr (MODE == RED_DOT_NORM) c += (double)norm2(yv.c[k]);
            }
        }
    }
    __shared__ double lds[BT / 64];
    constexpr int K = MODE == RED_NORM ? 1 : MODE == RED_DOT ? 2 : 3;
    double *out = partial + L.part * K;
    const double sa = block_sum<BT>(a, lds);
    if (threadIdx.x == 0) out[0] = sa;
    if constexpr (K >= 2) {
        const double sb = block_sum<BT>(b, lds);
        if (threadIdx.x == 0) out[1] = sb;
    }
    if constexpr (K == 3) {
        const double scc = block_sum<BT>(c, lds);
        if (threadIdx.x == 0) out[2] = scc;
    }
}

hipError_t launch_reduce(FieldView x, FieldView y, int mode, double *partial, hipStream_t s, const double *mask,
                         int sps)
{
    const dim3 grid = x.tiles ? dim3(x.ntiles) : dim3(blas_blocks(x.n), x.nrhs);
#define LQ_RED(P)                                                                                            \
    if (mode == RED_NORM) reduce_kernel<P, RED_NORM><<<grid, BT, 0, s>>>(x, y, partial, mask, sps);         \
    else if (mode == RED_DOT) reduce_kernel<P, RED_DOT><<<grid, BT, 0, s>>>(x, y, partial, mask, sps);      \
    else reduce_kernel<P, RED_DOT_NORM><<<grid, BT, 0, s>>>(x, y, partial, mask, sps);
    switch (x.prec) {
    case F64: LQ_RED(F64) break;
    case F32: LQ_RED(F32) break;
    case F16: LQ_RED(F16) break;
    default: return hipErrorInvalidValue;
    }
#undef LQ_RED
    return hipGetLastError();
}

// One workgroup of FT threads per system: sum K values over sps * nblocks
// partials in a fixed order, then update the system's scalars.
constexpr int FT = 1024;
__global__ __launch_bounds__(FT) void finish_kernel(const double *partial, int sps, int nblocks, int K, int op,
                                                   double *scal, double eps, const int2 *range)
{
    const int sys = blockIdx.x;
    // a system's partials: sps * nblocks of them in order, or (ragged) the
    // count range[sys].y starting at range[sys].x
    const long cnt = range ? (long)range[sys].y : (long)sps * nblocks;
    const double *p = partial + (range ? (long)range[sys].x : (long)sys * cnt) * K;
    double v[3] = {0, 0, 0};
    // each thread adds its partials j = tid, tid + FT, ... in that order;
    // the loads of 8 of them are issued together
    constexpr int U = 8;
    for (long j0 = threadIdx.x; j0 < cnt; j0 += U * FT) {
        double t[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long j = j0 + (long)u * FT;
#pragma unroll
            for (int k = 0; k < 3; ++k) t[u][k] = (j < cnt && k < K) ? p[j * K + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + (long)u * FT < cnt)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k < K) v[k] += t[u][k];
    }
    __shared__ double lds[FT / 64];
    double tot[3];
    for (int k = 0; k < 3; ++k) tot[k] = block_sum<FT>(v[k], lds);
    if (threadIdx.x != 0) return;
    double *sc = scal + (long)sys * NSC;
    const bool fz = frozen(sc);
    switch (op) {
    case FIN_NORM: {
        const double n2 = tot[0];
        sc[SC_NORM2] = n2;
        sc[SC_SCALE] = sqrt(n2);
        sc[SC_INVSCALE] = n2 > 0 ? 1.0 / sqrt(n2) : 0.0;
        sc[SC_ODONE] = (n2 <= sc[SC_OTARGET2]) ? 1.0 : 0.0;
        break;
    }
    case FIN_INIT_CG:
    case FIN_INIT_BICG: {
        const double rr = tot[0];
        sc[SC_RR] = rr;
        sc[SC_TARGET2] *= rr;  // relative -> absolute
        sc[SC_ITER] = 0;
        sc[SC_BREAK] = 0;
        sc[SC_DONE] = (sc[SC_ODONE] != 0.0 || rr <= sc[SC_TARGET2] || !(rr > 0)) ? 1.0 : 0.0;
        sc[SC_ALPHA_RE] = sc[SC_OMEGA_RE] = 1.0;
        sc[SC_ALPHA_IM] = sc[SC_OMEGA_IM] = 0.0;
        sc[SC_BETA_RE] = sc[SC_BETA_IM] = 0.0;
        sc[SC_RHO_RE] = rr;
        sc[SC_RHO_IM] = 0.0;
        break;
    }
    case FIN_CG_ALPHA: {
        const double den = tot[0];
        if (fz || !(den > 0)) {
            if (!fz) sc[SC_BREAK] = 1.0;
            sc[SC_ALPHA_RE] = 0.0;
        } else {
            sc[SC_ALPHA_RE] = sc[SC_RR] / den;
        }
        sc[SC_ALPHA_IM] = 0.0;
        break;
    }
    case FIN_CG_BETA: {
        const double rr = tot[0];
        if (fz) {
            sc[SC_BETA_RE] = 0.0;
        } else {
            sc[SC_BETA_RE] = rr / sc[SC_RR];
            sc[SC_RR_PREV] = sc[SC_RR];
            sc[SC_RR] = rr;
            sc[SC_ITER] += 1.0;
            if (rr <= sc[SC_TARGET2]) sc[SC_DONE] = 1.0;
            if (!(rr == rr) || rr > 1e300) sc[SC_BREAK] = 1.0;
        }
        sc[SC_BETA_IM] = 0.0;
        break;
    }
    case FIN_BICG_ALPHA: {
        // a frozen system keeps alpha and omega of its last iteration (a
        // reliable-update restart continues from them; no kernel reads the
        // scalars of a frozen system)
        if (fz) break;
        const double dr = tot[0], di = tot[1];
        const double d2 = dr * dr + di * di;
        if (!(d2 > 0) || !(d2 < 1e300)) {
            sc[SC_BREAK] = 1.0;
            sc[SC_ALPHA_RE] = sc[SC_ALPHA_IM] = 0.0;
        } else {
            const double rr_ = sc[SC_RHO_RE], ri = sc[SC_RHO_IM];
            sc[SC_ALPHA_RE] = (rr_ * dr + ri * di) / d2;
            sc[SC_ALPHA_IM] = (ri * dr - rr_ * di) / d2;
        }
        break;
    }
    case FIN_BICG_OMEGA: {
        // tot = <s, t> (re, im), |t|^2 ; omega = <t, s> / |t|^2 = conj(<s, t>) / |t|^2
        const double tt = tot[2];
        if (fz) break;
        if (!(tt > 0)) {
            sc[SC_OMEGA_RE] = sc[SC_OMEGA_IM] = 0.0;
        } else {
            sc[SC_OMEGA_RE] = tot[0] / tt;
            sc[SC_OMEGA_IM] = -tot[1] / tt;
        }
        break;
    }
    case FIN_BICG_RHO: {
        const bool forced = sc[SC_FORCE_BREAK] > 0 && sc[SC_ITER] + 1.0 == sc[SC_FORCE_BREAK];
        const double pr = forced ? 0.0 : tot[0], pi = forced ? 0.0 : tot[1], rr = tot[2];
        if (fz) {
            sc[SC_BETA_RE] = sc[SC_BETA_IM] = 0.0;
            break;
        }
        sc[SC_RR] = rr;
        sc[SC_ITER] += 1.0;
        if (rr <= sc[SC_TARGET2]) {
            sc[SC_DONE] = 1.0;
            sc[SC_BETA_RE] = sc[SC_BETA_IM] = 0.0;
            break;
        }
        const double om2 = sc[SC_OMEGA_RE] * sc[SC_OMEGA_RE] + sc[SC_OMEGA_IM] * sc[SC_OMEGA_IM];
        const double rho2 = sc[SC_RHO_RE] * sc[SC_RHO_RE] + sc[SC_RHO_IM] * sc[SC_RHO_IM];
        if (!(rr == rr) || !(om2 > 0) || !(rho2 > 0) || (pr * pr + pi * pi) < eps * eps * rr * rr) {
            sc[SC_BREAK] = 1.0;
            sc[SC_BETA_RE] = sc[SC_BETA_IM] = 0.0;
            break;
        }
        // beta = (rho_new / rho) * (alpha / omega)
        const double qr = (pr * sc[SC_RHO_RE] + pi * sc[SC_RHO_IM]) / rho2;
        const double qi = (pi * sc[SC_RHO_RE] - pr * sc[SC_RHO_IM]) / rho2;
        const double ar = (sc[SC_ALPHA_RE] * sc[SC_OMEGA_RE] + sc[SC_ALPHA_IM] * sc[SC_OMEGA_IM]) / om2;
        const double ai = (sc[SC_ALPHA_IM] * sc[SC_OMEGA_RE] - sc[SC_ALPHA_RE] * sc[SC_OMEGA_IM]) / om2;
        sc[SC_BETA_RE] = qr * ar - qi * ai;
        sc[SC_BETA_IM] = qr * ai + qi * ar;
        sc[SC_RHO_RE] = pr;
        sc[SC_RHO_IM] = pi;
        break;
    }
    case FIN_DOT:
        sc[SC_DOT_RE] = tot[0];
        sc[SC_DOT_IM] = tot[1];
        break;
    case FIN_BICG_RESTART:
    case FIN_CG_RESTART: {
        // the residual r was replaced by the true one, in the normalisation
        // of this inner solve; the stored scalars are those of the last
        // iteration before the replacement (its x and r update done, the
        // search direction not yet updated)
        const double rr = tot[2];
        const bool fresh = sc[SC_REINIT] != 0.0;
        sc[SC_TARGET2] *= rr;  // relative -> absolute
        sc[SC_ITER] = 0;
        sc[SC_BREAK] = 0;
        sc[SC_DONE] = (sc[SC_ODONE] != 0.0 || rr <= sc[SC_TARGET2] || !(rr > 0)) ? 1.0 : 0.0;
        double br = 0.0, bi = 0.0;
        if (op == FIN_CG_RESTART) {
            // p = r + beta (p - c r): the search direction first loses its
            // component along the replaced residual (c = <r, p> / |r|^2; in
            // exact arithmetic r is orthogonal to p), then beta = |r|^2 /
            // |r_old|^2 with |r_old|^2 and p taken into the new normalisation
            // (factors SC_RESCALE^2, SC_RESCALE).  tot = <p, r>, |r|^2.
            const double den = sc[SC_RESCALE] * sc[SC_RR_PREV];
            if (!fresh && den > 0 && den < 1e300 && rr > 0) {
                br = rr / den;
                sc[SC_OMEGA_RE] = tot[0] / rr;
                sc[SC_OMEGA_IM] = -tot[1] / rr;
            } else {
                sc[SC_OMEGA_RE] = sc[SC_OMEGA_IM] = 0.0;
            }
            sc[SC_ALPHA_RE] = sc[SC_ALPHA_IM] = 0.0;
        } else {
            // beta = (rho_new / rho) (alpha / omega) as in FIN_BICG_RHO; rho,
            // p and v change normalisation by the same factor, which cancels.
            // A fresh system, or one whose last scalars admit no
            // continuation, takes beta = 0 (p = r)
            const double pr = fresh ? rr : tot[0], pi = fresh ? 0.0 : tot[1];
            const double om2 = sc[SC_OMEGA_RE] * sc[SC_OMEGA_RE] + sc[SC_OMEGA_IM] * sc[SC_OMEGA_IM];
            const double rho2 = sc[SC_RHO_RE] * sc[SC_RHO_RE] + sc[SC_RHO_IM] * sc[SC_RHO_IM];
            if (!fresh && om2 > 0 && rho2 > 0 && om2 < 1e300 && rho2 < 1e300) {
                const double qr = (pr * sc[SC_RHO_RE] + pi * sc[SC_RHO_IM]) / rho2;
                const double qi = (pi * sc[SC_RHO_RE] - pr * sc[SC_RHO_IM]) / rho2;
                const double ar = (sc[SC_ALPHA_RE] * sc[SC_OMEGA_RE] + sc[SC_ALPHA_IM] * sc[SC_OMEGA_IM]) / om2;
                const double ai = (sc[SC_ALPHA_IM] * sc[SC_OMEGA_RE] - sc[SC_ALPHA_RE] * sc[SC_OMEGA_IM]) / om2;
                br = qr * ar - qi * ai;
                bi = qr * ai + qi * ar;
            }
            if (!(br == br) || !(bi == bi)) br = bi = 0.0;
            if (fresh) {
                sc[SC_ALPHA_RE] = sc[SC_OMEGA_RE] = 1.0;
                sc[SC_ALPHA_IM] = sc[SC_OMEGA_IM] = 0.0;
            }
            sc[SC_RHO_RE] = pr;
            sc[SC_RHO_IM] = pi;
        }
        if (!(br == br)) br = 0.0;
        sc[SC_BETA_RE] = br;
        sc[SC_BETA_IM] = bi;
        sc[SC_RR] = rr;
        break;
    }
    }
}

hipError_t launch_finish(const double *partial, int nsys, int sps, int nblocks, int K, int op, double *sc,
                         double eps, hipStream_t s, const int2 *range)
{
    finish_kernel<<<nsys, FT, 0, s>>>(partial, sps, nblocks, K, op, sc, eps, range);
    return hipGetLastError();
}

// ----------------------------------------------------------- elementwise --

#define LQ_SITE                                                 \
    const Loc L = locate(x);                                    \
    const long i = L.i;                                         \
    const int slice = L.slice;                                  \
    if (i >= L.n) return;

template <int P> __global__ __launch_bounds__(BT) void zero_kernel(FieldView x)
{
    using R = typename PT<P>::R;
    LQ_SITE
    Spinor<R> z;
#pragma unroll
    for (int k = 0; k < 12; ++k) z.c[k] = cx<R>{0, 0};
    store_spinor<P>(at(x, L), i, L.n, z);
}

template <int PY, int PX>
__global__ __launch_bounds__(BT) void copy_kernel(FieldView y, FieldView x, const double *sc, int sps, bool scaled)
{
    using RX = typename PT<PX>::R;
    using RY = typename PT<PY>::R;
    LQ_SITE
    const Spinor<RX> v = load_spinor<PX>(at(x, L), i, L.n);
    const double f = scaled ? sc[(slice / sps) * NSC + SC_INVSCALE] : 1.0;
    Spinor<RY> o;
#pragma unroll
    for (int k = 0; k < 12; ++k) o.c[k] = cx<RY>{(RY)(f * (double)v.c[k].re), (RY)(f * (double)v.c[k].im)};
    store_spinor<PY>(at(y, L), i, L.n, o);
}

template <int PE>
__global__ __launch_bounds__(BT) void accum_kernel(FieldView x, FieldView e, const double *sc, int sps, bool scaled)
{
    using RE = typename PT<PE>::R;
    LQ_SITE
    const double *s = sc + (slice / sps) * NSC;
    if (s[SC_ODONE] != 0.0) return;
    const double f = scaled ? s[SC_SCALE] : 1.0;
    Spinor<double> xv = load_spinor<F64>(at(x, L), i, L.n);
    const Spinor<RE> ev = load_spinor<PE>(at(e, L), i, L.n);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        xv.c[k].re += f * (double)ev.c[k].re;
        xv.c[k].im += f * (double)ev.c[k].im;
    }
    store_spinor<F64>(at(x, L), i, L.n, xv);
}

__global__ __launch_bounds__(BT) void xmy_norm_kernel(FieldView r, FieldView b, FieldView x /* y */,
                                                     double *partial)
{
    const Loc L = locate(r);
    const long i = L.i;
    double a = 0;
    if (i < L.n) {
        const Spinor<double> bv = load_spinor<F64>(at(b, L), i, L.n);
        const Spinor<double> yv = load_spinor<F64>(at(x, L), i, L.n);
        Spinor<double> o;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            o.c[k] = bv.c[k] - yv.c[k];
            a += norm2(o.c[k]);
        }
        store_spinor<F64>(at(r, L), i, L.n, o);
    }
    __shared__ double lds[BT / 64];
    const double t = block_sum<BT>(a, lds);
    if (threadIdx.x == 0) partial[L.part] = t;
}

// r -= sc[SC_SCALE] e (systems with SC_ODONE set keep r) and partial |r|^2
template <int PE>
__global__ __launch_bounds__(BT) void sub_scaled_norm_kernel(FieldView r, FieldView e, const double *sc, int sps,
                                                            double *partial)
{
    using RE = typename PT<PE>::R;
    const Loc L = locate(r);
    const long i = L.i;
    const int slice = L.slice;
    const double *s = sc + (slice / sps) * NSC;
    const double f = s[SC_ODONE] != 0.0 ? 0.0 : s[SC_SCALE];
    double a = 0;
    if (i < L.n) {
        Spinor<double> rv = load_spinor<F64>(at(r, L), i, L.n);
        const Spinor<RE> ev = load_spinor<PE>(at(e, L), i, L.n);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            rv.c[k].re -= f * (double)ev.c[k].re;
            rv.c[k].im -= f * (double)ev.c[k].im;
            a += norm2(rv.c[k]);
        }
        store_spinor<F64>(at(r, L), i, L.n, rv);
    }
    __shared__ double lds[BT / 64];
    const double t = block_sum<BT>(a, lds);
    if (threadIdx.x == 0) partial[L.part] = t;
}

template <int P, int PX>
__global__ __launch_bounds__(BT) void cg_xr_kernel(FieldView x, FieldView r, FieldView p, FieldView q,
                                                  const double *sc, int sps, double *partial)
{
    using R = typename PT<P>::R;
    using RX = typename PT<PX>::R;
    const Loc L = locate(r);
    const long i = L.i;
    const int slice = L.slice;
    const double *s = sc + (slice / sps) * NSC;
    double a = 0;
    if (i < L.n && !frozen(s)) {
        Spinor<R> rv = load_spinor<P>(at(r, L), i, L.n);
        {
            const R al = (R)s[SC_ALPHA_RE];
            const Spinor<R> pv = load_spinor<P>(at(p, L), i, L.n);
            const Spinor<R> qv = load_spinor<P>(at(q, L), i, L.n);
            Spinor<RX> xv = load_spinor<PX>(at(x, L), i, L.n);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                xv.c[k].re += (RX)(al * pv.c[k].re);
                xv.c[k].im += (RX)(al * pv.c[k].im);
                rv.c[k] = rv.c[k] - al * qv.c[k];
            }
            store_spinor<PX>(at(x, L), i, L.n, xv);
            store_spinor<P>(at(r, L), i, L.n, rv);
            rv = as_stored<P>(rv);  // the values as stored (binary16: rounded and scaled), not re-read
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) a += (double)norm2(rv.c[k]);
    }
    __shared__ double lds[BT / 64];
    const double t = block_sum<BT>(a, lds);
    if (threadIdx.x == 0) partial[L.part] = t;
}

template <int P>
__global__ __launch_bounds__(BT) void cg_p_kernel(FieldView p, FieldView x /* r */, const double *sc, int sps)
{
    using R = typename PT<P>::R;
    LQ_SITE
    const double *s = sc + (slice / sps) * NSC;
    if (frozen(s)) return;
    const R be = (R)s[SC_BETA_RE];
    const Spinor<R> rv = load_spinor<P>(at(x, L), i, L.n);
    Spinor<R> pv = load_spinor<P>(at(p, L), i, L.n);
#pragma unroll
    for (int k = 0; k < 12; ++k) pv.c[k] = rv.c[k] + be * pv.c[k];
    store_spinor<P>(at(p, L), i, L.n, pv);
}

template <int P>
__global__ __launch_bounds__(BT) void bicg_s_kernel(FieldView sv, FieldView x /* r */, FieldView v, const double *sc,
                                                   int sps)
{
    using R = typename PT<P>::R;
    LQ_SITE
    const double *s = sc + (slice / sps) * NSC;
    if (frozen(s)) return;
    const cx<R> al = scal<R>(s, SC_ALPHA_RE);
    const Spinor<R> rv = load_spinor<P>(at(x, L), i, L.n);
    const Spinor<R> vv = load_spinor<P>(at(v, L), i, L.n);
    Spinor<R> o;
#pragma unroll
    for (int k = 0; k < 12; ++k) o.c[k] = rv.c[k] - al * vv.c[k];
    store_spinor<P>(at(sv, L), i, L.n, o);
}

template <int P, int PX>
__global__ __launch_bounds__(BT) void bicg_xr_kernel(FieldView x, FieldView r, FieldView p, FieldView sv, FieldView t,
                                                    FieldView rhat, const double *sc, int sps, double *partial)
{
    using R = typename PT<P>::R;
    using RX = typename PT<PX>::R;
    const Loc L = locate(r);
    const long i = L.i;
    const int slice = L.slice;
    const double *s = sc + (slice / sps) * NSC;
    double a = 0, b = 0, c = 0;
    if (i < L.n) {
        Spinor<R> rv;
        if (!frozen(s)) {
            const cx<R> al = scal<R>(s, SC_ALPHA_RE);
            const cx<R> om = scal<R>(s, SC_OMEGA_RE);
            const Spinor<R> pv = load_spinor<P>(at(p, L), i, L.n);
            const Spinor<R> svv = load_spinor<P>(at(sv, L), i, L.n);
            const Spinor<R> tv = load_spinor<P>(at(t, L), i, L.n);
            Spinor<RX> xv = load_spinor<PX>(at(x, L), i, L.n);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cx<R> d = al * pv.c[k] + om * svv.c[k];
                xv.c[k].re += (RX)d.re;
                xv.c[k].im += (RX)d.im;
                rv.c[k] = svv.c[k] - om * tv.c[k];
            }
            store_spinor<PX>(at(x, L), i, L.n, xv);
            store_spinor<P>(at(r, L), i, L.n, rv);
            rv = as_stored<P>(rv);  // the values as stored (binary16: rounded and scaled), not re-read
            const Spinor<R> hv = load_spinor<P>(at(rhat, L), i, L.n);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const cx<R> d = cmulc(hv.c[k], rv.c[k]);
                a += (double)d.re;
                b += (double)d.im;
                c += (double)norm2(rv.c[k]);
            }
        }
    }
    __shared__ double lds[BT / 64];
    double *out = partial + L.part * 3;
    const double sa = block_sum<BT>(a, lds);
    const double sb = block_sum<BT>(b, lds);
    const double scc = block_sum<BT>(c, lds);
    if (threadIdx.x == 0) {
        out[0] = sa;
        out[1] = sb;
        out[2] = scc;
    }
}

template <int P>
__global__ __launch_bounds__(BT) void bicg_p_kernel(FieldView p, FieldView x /* r */, FieldView v, const double *sc,
                                                   int sps)
{
    using R = typename PT<P>::R;
    LQ_SITE
    const double *s = sc + (slice / sps) * NSC;
    if (frozen(s)) return;
    const cx<R> be = scal<R>(s, SC_BETA_RE);
    const cx<R> om = scal<R>(s, SC_OMEGA_RE);
    const Spinor<R> rv = load_spinor<P>(at(x, L), i, L.n);
    const Spinor<R> vv = load_spinor<P>(at(v, L), i, L.n);
    Spinor<R> pv = load_spinor<P>(at(p, L), i, L.n);
#pragma unroll
    for (int k = 0; k < 12; ++k) pv.c[k] = rv.c[k] + be * (pv.c[k] - om * vv.c[k]);
    store_spinor<P>(at(p, L), i, L.n, pv);
}

// a = src, b = src, z = 0 on the systems starting a new Krylov space (all
// operands in precision P; b and z optional)
template <int P>
__global__ __launch_bounds__(BT) void reinit_kernel(FieldView a, FieldView b, FieldView z, FieldView x /* src */,
                                                   const double *sc, int sps)
{
    using R = typename PT<P>::R;
    LQ_SITE
    const double *s = sc + (slice / sps) * NSC;
    if (s[SC_REINIT] == 0.0 || s[SC_ODONE] != 0.0) return;
    const Spinor<R> v = load_spinor<P>(at(x, L), i, L.n);
    store_spinor<P>(at(a, L), i, L.n, v);
    if (b.base) store_spinor<P>(at(b, L), i, L.n, v);
    if (z.base) {
        Spinor<R> o;
#pragma unroll
        for (int k = 0; k < 12; ++k) o.c[k] = cx<R>{0, 0};
        store_spinor<P>(at(z, L), i, L.n, o);
    }
}

template <int P> __global__ __launch_bounds__(BT) void gamma5_kernel(FieldView x)
{
    using R = typename PT<P>::R;
    LQ_SITE
    Spinor<R> v = load_spinor<P>(at(x, L), i, L.n);
#pragma unroll
    for (int k = 6; k < 12; ++k) v.c[k] = cx<R>{-v.c[k].re, -v.c[k].im};
    store_spinor<P>(at(x, L), i, L.n, v);
}

#undef LQ_SITE

static dim3 grid_of(const FieldView &x) { return x.tiles ? dim3(x.ntiles) : dim3(blas_blocks(x.n), x.nrhs); }

#define LQ_BY_PREC(prec, KER, ...)                                                    \
    switch (prec) {                                                                   \
    case F64: KER<F64><<<grid_of(x), BT, 0, s>>>(__VA_ARGS__); break;                 \
    case F32: KER<F32><<<grid_of(x), BT, 0, s>>>(__VA_ARGS__); break;                 \
    case F16: KER<F16><<<grid_of(x), BT, 0, s>>>(__VA_ARGS__); break;                 \
    default: return hipErrorInvalidValue;                                             \
    }                                                                                 \
    return hipGetLastError();

hipError_t launch_zero(FieldView x, hipStream_t s) { LQ_BY_PREC(x.prec, zero_kernel, x) }

hipError_t launch_reinit(FieldView a, FieldView b, FieldView z, FieldView x, const double *sc, int sps,
                         hipStream_t s)
{
    if (a.prec != x.prec || (b.base && b.prec != x.prec) || (z.base && z.prec != x.prec)) return hipErrorInvalidValue;
    LQ_BY_PREC(x.prec, reinit_kernel, a, b, z, x, sc, sps)
}

hipError_t launch_copy(FieldView y, FieldView x, const double *sc, int sps, bool scaled, hipStream_t s)
{
    const dim3 g = grid_of(x);
#define LQ_CP(PY, PX)                                                           \
    if (y.prec == PY && x.prec == PX) {                                         \
        copy_kernel<PY, PX><<<g, BT, 0, s>>>(y, x, sc, sps, scaled);            \
        return hipGetLastError();                                               \
    }
    LQ_CP(F64, F64) LQ_CP(F32, F64) LQ_CP(F16, F64) LQ_CP(F32, F32) LQ_CP(F16, F16) LQ_CP(F64, F32)
    LQ_CP(F32, F16) LQ_CP(F16, F32)
#undef LQ_CP
    return hipErrorInvalidValue;
}

hipError_t launch_accum(FieldView x64, FieldView e, const double *sc, int sps, bool scaled, hipStream_t s)
{
    FieldView &x = x64;
    LQ_BY_PREC(e.prec, accum_kernel, x64, e, sc, sps, scaled)
}

hipError_t launch_sub_scaled_norm(FieldView r, FieldView e, const double *sc, int sps, double *partial,
                                  hipStream_t s)
{
    FieldView &x = r;
    LQ_BY_PREC(e.prec, sub_scaled_norm_kernel, r, e, sc, sps, partial)
}

hipError_t launch_xmy_norm(FieldView r, FieldView b, FieldView y, double *partial, hipStream_t s)
{
    xmy_norm_kernel<<<grid_of(r), BT, 0, s>>>(r, b, y, partial);
    return hipGetLastError();
}

hipError_t launch_cg_xr(FieldView x, FieldView r, FieldView p, FieldView q, const double *sc, int sps,
                        double *partial, hipStream_t s)
{
    const dim3 g = grid_of(r);
    if (r.prec == F64 && x.prec == F64) cg_xr_kernel<F64, F64><<<g, BT, 0, s>>>(x, r, p, q, sc, sps, partial);
    else if (r.prec == F32 && x.prec == F32) cg_xr_kernel<F32, F32><<<g, BT, 0, s>>>(x, r, p, q, sc, sps, partial);
    else if (r.prec == F16 && x.prec == F32) cg_xr_kernel<F16, F32><<<g, BT, 0, s>>>(x, r, p, q, sc, sps, partial);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_cg_p(FieldView p, FieldView r, const double *sc, int sps, hipStream_t s)
{
    FieldView &x = r;
    LQ_BY_PREC(p.prec, cg_p_kernel, p, r, sc, sps)
}

hipError_t launch_bicg_s(FieldView sv, FieldView r, FieldView v, const double *sc, int sps, hipStream_t s)
{
    FieldView &x = r;
    LQ_BY_PREC(r.prec, bicg_s_kernel, sv, r, v, sc, sps)
}

hipError_t launch_bicg_xr(FieldView x, FieldView r, FieldView p, FieldView sv, FieldView t, FieldView rhat,
                          const double *sc, int sps, double *partial, hipStream_t s)
{
    const dim3 g = grid_of(r);
    if (r.prec == F64 && x.prec == F64)
        bicg_xr_kernel<F64, F64><<<g, BT, 0, s>>>(x, r, p, sv, t, rhat, sc, sps, partial);
    else if (r.prec == F32 && x.prec == F32)
        bicg_xr_kernel<F32, F32><<<g, BT, 0, s>>>(x, r, p, sv, t, rhat, sc, sps, partial);
    else if (r.prec == F16 && x.prec == F32)
        bicg_xr_kernel<F16, F32><<<g, BT, 0, s>>>(x, r, p, sv, t, rhat, sc, sps, partial);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_bicg_p(FieldView p, FieldView r, FieldView v, const double *sc, int sps, hipStream_t s)
{
    FieldView &x = r;
    LQ_BY_PREC(r.prec, bicg_p_kernel, p, r, v, sc, sps)
}

hipError_t launch_gamma5(FieldView x, hipStream_t s) { LQ_BY_PREC(x.prec, gamma5_kernel, x) }

#undef LQ_BY_PREC

}  // namespace lq
