// fields.hip -- field import/export, link packing and the clover term.
#include "fields.h"
#include "su3.h"
#include "stencil.h"

namespace lq {

// lexicographic site index of (p, cb)
__device__ __forceinline__ long lex_of(const Geom &g, int p, int cb)
{
    int c[4];
    cb_coords(g, p, cb, c);
    return c[0] + (long)g.L[0] * (c[1] + (long)g.L[1] * (c[2] + (long)g.L[2] * c[3]));
}

// ------------------------------------------------------------- spinors --

template <int P>
__global__ __launch_bounds__(256) void pack_spinor_kernel(Geom g, int p, int mode, const double *__restrict__ src,
                                                          FieldView dst)
{
    using R = typename PT<P>::R;
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int rhs = blockIdx.y;
    if (cb >= g.vh) return;
    const long vol = 2L * g.vh;
    const long site = mode == 0 ? lex_of(g, p, cb) : cb;
    const double *s = src + ((long)rhs * (mode == 0 ? vol : g.vh) + site) * 24;
    Spinor<R> v;
#pragma unroll
    for (int i = 0; i < 12; ++i) v.c[i] = cx<R>{(R)s[2 * i], (R)s[2 * i + 1]};
    store_spinor<P>(dst.base + rhs * dst.rs, cb, dst.n, v);
}

template <int P>
__global__ __launch_bounds__(256) void unpack_spinor_kernel(Geom g, int p, int mode, FieldView src,
                                                            double *__restrict__ dst)
{
    using R = typename PT<P>::R;
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int rhs = blockIdx.y;
    if (cb >= g.vh) return;
    const long vol = 2L * g.vh;
    const long site = mode == 0 ? lex_of(g, p, cb) : cb;
    double *d = dst + ((long)rhs * (mode == 0 ? vol : g.vh) + site) * 24;
    const Spinor<R> v = load_spinor<P>(src.base + rhs * src.rs, cb, src.n);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        d[2 * i] = (double)v.c[i].re;
        d[2 * i + 1] = (double)v.c[i].im;
    }
}

hipError_t launch_pack_spinor(const Geom &g, int p, int mode, const double *src, FieldView dst, hipStream_t s)
{
    const dim3 grid((g.vh + 255) / 256, dst.nrhs);
    switch (dst.prec) {
    case F64: pack_spinor_kernel<F64><<<grid, 256, 0, s>>>(g, p, mode, src, dst); break;
    case F32: pack_spinor_kernel<F32><<<grid, 256, 0, s>>>(g, p, mode, src, dst); break;
    case F16: pack_spinor_kernel<F16><<<grid, 256, 0, s>>>(g, p, mode, src, dst); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geom &g, int p, int mode, FieldView src, double *dst, hipStream_t s)
{
    const dim3 grid((g.vh + 255) / 256, src.nrhs);
    switch (src.prec) {
    case F64: unpack_spinor_kernel<F64><<<grid, 256, 0, s>>>(g, p, mode, src, dst); break;
    case F32: unpack_spinor_kernel<F32><<<grid, 256, 0, s>>>(g, p, mode, src, dst); break;
    case F16: unpack_spinor_kernel<F16><<<grid, 256, 0, s>>>(g, p, mode, src, dst); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// --------------------------------------------------------------- links --

__global__ __launch_bounds__(256) void pack_links_kernel(Geom g, const double *__restrict__ U, char *links64)
{
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int p = blockIdx.y;
    if (cb >= g.vh) return;
    const long site = lex_of(g, p, cb);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const double *u = U + (site * 4 + mu) * 18;
        double raw[18];
#pragma unroll
        for (int i = 0; i < 18; ++i) raw[i] = u[i];
        store_planes<double, 18>(links64 + (long)(p * 4 + mu) * link_bytes(F64, 18, g.vh), cb, g.vh, raw);
    }
}

template <int P, int NL>
__global__ __launch_bounds__(256) void convert_links_kernel(Geom g, const char *links64, char *dst)
{
    using S = typename PT<P>::S;
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int pm = blockIdx.y;  // parity * 4 + mu
    if (cb >= g.vh) return;
    double raw[18];
    load_planes<double, 18>(links64 + (long)pm * link_bytes(F64, 18, g.vh), cb, g.vh, raw);
    S o[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) o[i] = (S)raw[i];
    store_planes<S, NL>(dst + (long)pm * link_bytes(P, NL, g.vh), cb, g.vh, o);
}

hipError_t launch_pack_links_f64(const Geom &g, const double *U, char *links64, hipStream_t s)
{
    pack_links_kernel<<<dim3((g.vh + 255) / 256, 2), 256, 0, s>>>(g, U, links64);
    return hipGetLastError();
}

hipError_t launch_convert_links(const Geom &g, const char *links64, int prec, int nl, char *dst, hipStream_t s)
{
    const dim3 grid((g.vh + 255) / 256, 8);
    if (prec == F64 && nl == 12) convert_links_kernel<F64, 12><<<grid, 256, 0, s>>>(g, links64, dst);
    else if (prec == F32 && nl == 18) convert_links_kernel<F32, 18><<<grid, 256, 0, s>>>(g, links64, dst);
    else if (prec == F32 && nl == 12) convert_links_kernel<F32, 12><<<grid, 256, 0, s>>>(g, links64, dst);
    else if (prec == F16 && nl == 18) convert_links_kernel<F16, 18><<<grid, 256, 0, s>>>(g, links64, dst);
    else if (prec == F16 && nl == 12) convert_links_kernel<F16, 12><<<grid, 256, 0, s>>>(g, links64, dst);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// -------------------------------------------------------------- clover --

// t * U or t * U^dag for a link U loaded just before use (keeps one link
// and one partial product live at a time).
__device__ __forceinline__ M3 mul_link(const M3 &t, const Geom &g, const char *links64, const int c[4], int mu,
                                       bool dagger)
{
    const M3 u = link_at(g, links64, c, mu);
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (dagger)
                r.e[i * 3 + j] = t.e[i * 3 + 0] * conj(u.e[j * 3 + 0]) + t.e[i * 3 + 1] * conj(u.e[j * 3 + 1]) +
                                 t.e[i * 3 + 2] * conj(u.e[j * 3 + 2]);
            else
                r.e[i * 3 + j] = t.e[i * 3 + 0] * u.e[0 * 3 + j] + t.e[i * 3 + 1] * u.e[1 * 3 + j] +
                                 t.e[i * 3 + 2] * u.e[2 * 3 + j];
        }
    return r;
}

// One leaf: the product of four links along a closed path from x, each
// given by its start site, direction and whether it is walked backwards.
__device__ __forceinline__ M3 leaf(const Geom &g, const char *links64, const int *s0, int d0, bool b0, const int *s1,
                                   int d1, bool b1, const int *s2, int d2, bool b2, const int *s3, int d3, bool b3)
{
    M3 t;
#pragma unroll
    for (int i = 0; i < 9; ++i) t.e[i] = cx<double>{(i % 4) == 0 ? 1.0 : 0.0, 0.0};
    t = mul_link(t, g, links64, s0, d0, b0);
    t = mul_link(t, g, links64, s1, d1, b1);
    t = mul_link(t, g, links64, s2, d2, b2);
    t = mul_link(t, g, links64, s3, d3, b3);
    return t;
}

// Fhat_{mu nu}(x) = (Q - Q^dag)/8 from the four counter-clockwise leaves;
// colour trace removed if traceless.
__device__ M3 field_strength(const Geom &g, const char *links64, const int c[4], int mu, int nu, int traceless)
{
    int pm[4], pn[4], mm[4], mn[4], mmpn[4], mmmn[4], pmmn[4];
    shift(g, c, mu, 1, nu, 0, pm);     // x + mu
    shift(g, c, mu, 0, nu, 1, pn);     // x + nu
    shift(g, c, mu, -1, nu, 0, mm);    // x - mu
    shift(g, c, mu, 0, nu, -1, mn);    // x - nu
    shift(g, c, mu, -1, nu, 1, mmpn);  // x - mu + nu
    shift(g, c, mu, -1, nu, -1, mmmn); // x - mu - nu
    shift(g, c, mu, 1, nu, -1, pmmn);  // x + mu - nu
    // (+mu, +nu): U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    M3 Q = leaf(g, links64, c, mu, false, pm, nu, false, pn, mu, true, c, nu, true);
    // (-mu, +nu): U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
    M3 t = leaf(g, links64, c, nu, false, mmpn, mu, true, mm, nu, true, mm, mu, false);
#pragma unroll
    for (int i = 0; i < 9; ++i) Q.e[i] = Q.e[i] + t.e[i];
    // (-mu, -nu): U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
    t = leaf(g, links64, mm, mu, true, mmmn, nu, true, mmmn, mu, false, mn, nu, false);
#pragma unroll
    for (int i = 0; i < 9; ++i) Q.e[i] = Q.e[i] + t.e[i];
    // (+mu, -nu): U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
    t = leaf(g, links64, mn, nu, true, mn, mu, false, pmmn, nu, false, c, mu, true);
#pragma unroll
    for (int i = 0; i < 9; ++i) Q.e[i] = Q.e[i] + t.e[i];
    M3 F;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) F.e[i * 3 + j] = 0.125 * (Q.e[i * 3 + j] - conj(Q.e[j * 3 + i]));
    if (traceless) {
        const cx<double> tr = (1.0 / 3.0) * (F.e[0] + F.e[4] + F.e[8]);
        F.e[0] = F.e[0] - tr;
        F.e[4] = F.e[4] - tr;
        F.e[8] = F.e[8] - tr;
    }
    return F;
}

// In the chiral basis gamma_k gamma_l (k < l spatial) = diag(i eps_klm sigma_m)
// on both chiral halves and gamma_k gamma_t = diag(-i sigma_k, +i sigma_k).
// With eta = -1 (spins 0,1) or +1 (spins 2,3),
//   X = F_yz + eta F_xt,  Y = F_xz - eta F_yt,  Z = F_xy + eta F_zt,
// the block of sum_{mu<nu} gamma_mu gamma_nu (x) F_{mu nu} is
//   [[ i Z, i X - Y ], [ i X + Y, -i Z ]]   (2x2 spin blocks of 3x3 colour),
// and the clover block is A = 1 - c_sw kappa times it.  The blocks are
// linear in the F_{mu nu}, so they are accumulated one plane at a time:
// add_plane adds one plane's field strength F to both packed blocks
// o[0..35], o[36..71] (6 diagonal reals, then the 15 strictly-lower entries
// row by row as (re, im)); WHICH says whether F enters X (0), Y (1) or Z (2),
// c0 / c1 is its factor (-c_sw kappa times the sign) in each block.
template <int WHICH>
__device__ __forceinline__ void add_plane(double o[72], const M3 &F, double c0, double c1)
{
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        double *ob = o + 36 * b;
        const double cf = b == 0 ? c0 : c1;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const cx<double> f = cf * F.e[a * 3 + d];
                if constexpr (WHICH != 2) {
                    // lower-left 3x3: entry (3 + a, d)
                    const cx<double> v = WHICH == 0 ? ti(f) : f;
                    const int k = 6 + 2 * ((3 + a) * (2 + a) / 2 + d);
                    ob[k] += v.re;
                    ob[k + 1] += v.im;
                } else if (a == d) {
                    ob[a] += ti(f).re;
                    ob[3 + a] += tmi(f).re;
                } else if (a > d) {
                    const int k1 = 6 + 2 * (a * (a - 1) / 2 + d);
                    const int k2 = 6 + 2 * ((3 + a) * (2 + a) / 2 + 3 + d);
                    ob[k1] += ti(f).re;
                    ob[k1 + 1] += ti(f).im;
                    ob[k2] += tmi(f).re;
                    ob[k2 + 1] += tmi(f).im;
                }
            }
    }
}

// The six planes in the order the blocks are assembled: (mu, nu), whether
// the plane enters X (0), Y (1) or Z (2), and its sign in the second block
// relative to the first (eta = -1, +1 for the two chirality blocks).
__device__ __forceinline__ void plane_of(int pl, int &mu, int &nu)
{
    switch (pl) {
    case 0: mu = 0; nu = 1; break;  // Z: F_xy
    case 1: mu = 2; nu = 3; break;  // Z: eta F_zt
    case 2: mu = 1; nu = 2; break;  // X: F_yz
    case 3: mu = 0; nu = 3; break;  // X: eta F_xt
    case 4: mu = 0; nu = 2; break;  // Y: F_xz
    default: mu = 1; nu = 3; break; // Y: -eta F_yt
    }
}

// One (site, plane) per thread: Fhat_{mu nu}(x) into fbuf
// [parity][plane][18 reals over vh].
__global__ __launch_bounds__(128) void field_strength_kernel(Geom g, const char *links64, int traceless, char *fbuf)
{
    const int cb = blockIdx.x * 128 + threadIdx.x;
    const int pl = blockIdx.y;
    const int p = blockIdx.z;
    if (cb >= g.vh) return;
    int c[4], mu, nu;
    cb_coords(g, p, cb, c);
    plane_of(pl, mu, nu);
    const M3 F = field_strength(g, links64, c, mu, nu, traceless);
    double raw[18];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        raw[2 * i] = F.e[i].re;
        raw[2 * i + 1] = F.e[i].im;
    }
    store_planes<double, 18>(fbuf + (long)(p * 6 + pl) * Planes<double, 18>::field_bytes(g.vh), cb, g.vh, raw);
}

__device__ __forceinline__ M3 plane_at(const Geom &g, const char *fbuf, int p, int pl, int cb)
{
    double raw[18];
    load_planes<double, 18>(fbuf + (long)(p * 6 + pl) * Planes<double, 18>::field_bytes(g.vh), cb, g.vh, raw);
    M3 m;
#pragma unroll
    for (int i = 0; i < 9; ++i) m.e[i] = cx<double>{raw[2 * i], raw[2 * i + 1]};
    return m;
}

// One site per thread: A = 1 + F assembled from the six field strengths.
__global__ __launch_bounds__(128) void clover_build_kernel(Geom g, const char *fbuf, double csw, double kappa,
                                                          char *clov64)
{
    const int cb = blockIdx.x * 128 + threadIdx.x;
    const int p = blockIdx.y;
    if (cb >= g.vh) return;
    double o[72];
#pragma unroll
    for (int i = 0; i < 72; ++i) o[i] = (i % 36) < 6 ? 1.0 : 0.0;
    const double ck = -csw * kappa;
    add_plane<2>(o, plane_at(g, fbuf, p, 0, cb), ck, ck);
    add_plane<2>(o, plane_at(g, fbuf, p, 1, cb), -ck, ck);
    add_plane<0>(o, plane_at(g, fbuf, p, 2, cb), ck, ck);
    add_plane<0>(o, plane_at(g, fbuf, p, 3, cb), -ck, ck);
    add_plane<1>(o, plane_at(g, fbuf, p, 4, cb), ck, ck);
    add_plane<1>(o, plane_at(g, fbuf, p, 5, cb), ck, -ck);
    store_planes<double, 72>(clov64 + (long)p * clover_bytes(F64, g.vh), cb, g.vh, o);
}

// One 6x6 Hermitian block per thread, inverted in place by Gauss-Jordan
// elimination with partial (row) pivoting; the row exchanges are undone as
// column exchanges at the end.  The 64 blocks of a workgroup live in LDS as
// [row][col][thread], so the pivot row can be indexed at run time without
// private (scratch) memory and consecutive threads hit consecutive banks.
// The lower triangle of the inverse is packed as the Hermitian average of
// the two triangles.  Only the blocks of parity p are inverted.
constexpr int INV_T = 64;
__global__ __launch_bounds__(INV_T) void clover_invert_kernel(Geom g, int p, const char *clov64, char *inv64,
                                                             int *flag)
{
    __shared__ cx<double> lds[36 * INV_T];
    const int idx = blockIdx.x * INV_T + threadIdx.x;
    if (idx >= 2 * g.vh) return;  // every thread works on its own LDS column only
    const int cb = idx >> 1, b = idx & 1;
    cx<double> *a = lds + threadIdx.x;  // a[(i * 6 + j) * INV_T] is entry (i, j)
    auto at = [&](int i, int j) -> cx<double> & { return a[(i * 6 + j) * INV_T]; };
    const char *base = clov64 + (long)p * clover_bytes(F64, g.vh);
    double c[36];
    load_planes<double, 36, false, 576>(base + (long)18 * b * 16 * SB, cb, g.vh, c);
    double scale = 0.0;
    for (int i = 0; i < 6; ++i) {
        at(i, i) = cx<double>{c[i], 0.0};
        scale = fmax(scale, fabs(c[i]));
    }
    int k = 6;
    for (int i = 1; i < 6; ++i)
        for (int j = 0; j < i; ++j) {
            at(i, j) = cx<double>{c[k], c[k + 1]};
            at(j, i) = cx<double>{c[k], -c[k + 1]};
            scale = fmax(scale, sqrt(c[k] * c[k] + c[k + 1] * c[k + 1]));
            k += 2;
        }
    int perm[6];
    bool sing = false;
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        double best = norm2(at(col, col));
        for (int r = col + 1; r < 6; ++r) {
            const double v = norm2(at(r, col));
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        perm[col] = piv;
        if (!(sqrt(best) > 1e-14 * scale)) {
            sing = true;
            break;
        }
        if (piv != col)
            for (int j = 0; j < 6; ++j) {
                const cx<double> t = at(col, j);
                at(col, j) = at(piv, j);
                at(piv, j) = t;
            }
        const cx<double> pv = at(col, col);
        const double d = norm2(pv);
        const cx<double> inv = cx<double>{pv.re / d, -pv.im / d};
        at(col, col) = cx<double>{1.0, 0.0};
        for (int j = 0; j < 6; ++j) at(col, j) = inv * at(col, j);
        for (int r = 0; r < 6; ++r) {
            if (r == col) continue;
            const cx<double> f = at(r, col);
            at(r, col) = cx<double>{0.0, 0.0};
            for (int j = 0; j < 6; ++j) at(r, j) = at(r, j) - f * at(col, j);
        }
    }
    if (sing) {
        atomicOr(flag, 1);
    } else {
        for (int col = 5; col >= 0; --col)
            if (perm[col] != col)
                for (int i = 0; i < 6; ++i) {
                    const cx<double> t = at(i, col);
                    at(i, col) = at(i, perm[col]);
                    at(i, perm[col]) = t;
                }
    }
    double o[36];
    for (int i = 0; i < 6; ++i) o[i] = sing ? 0.0 : at(i, i).re;
    k = 6;
    for (int i = 1; i < 6; ++i)
        for (int j = 0; j < i; ++j) {
            o[k++] = sing ? 0.0 : 0.5 * (at(i, j).re + at(j, i).re);
            o[k++] = sing ? 0.0 : 0.5 * (at(i, j).im - at(j, i).im);
        }
    // block b owns planes 18b .. 18b + 17 of the site record (72 FP64 reals)
    char *dst = inv64 + (long)p * clover_bytes(F64, g.vh);
    store_planes<double, 36, false, 576>(dst + (long)18 * b * 16 * SB, cb, g.vh, o);
}

template <int P>
__global__ __launch_bounds__(256) void convert_clover_kernel(Geom g, int p0, const char *clov64, char *dst)
{
    using S = typename PT<P>::S;
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int p = p0 + blockIdx.y;
    if (cb >= g.vh) return;
    double raw[72];
    load_planes<double, 72>(clov64 + (long)p * clover_bytes(F64, g.vh), cb, g.vh, raw);
    S o[72];
#pragma unroll
    for (int i = 0; i < 72; ++i) o[i] = (S)raw[i];
    store_planes<S, 72>(dst + (long)p * clover_bytes(P, g.vh), cb, g.vh, o);
}

template <int P>
__global__ __launch_bounds__(256) void clover_apply_kernel(Geom g, const char *clov, FieldView out, FieldView in)
{
    using R = typename PT<P>::R;
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int rhs = blockIdx.y;
    if (cb >= g.vh) return;
    Spinor<R> v = load_spinor<P>(in.base + rhs * in.rs, cb, in.n);
    clover_mul<P>(clov, g.vh, cb, v);
    store_spinor<P>(out.base + rhs * out.rs, cb, out.n, v);
}

template <int P>
__global__ __launch_bounds__(256) void twist_apply_kernel(Geom g, double c_re, double c_im, FieldView out, FieldView in)
{
    using R = typename PT<P>::R;
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int rhs = blockIdx.y;
    if (cb >= g.vh) return;
    Spinor<R> v = load_spinor<P>(in.base + rhs * in.rs, cb, in.n);
    const cx<R> c = cx<R>{(R)c_re, (R)c_im};
#pragma unroll
    for (int i = 0; i < 6; ++i) v.c[i] = c * v.c[i];
#pragma unroll
    for (int i = 6; i < 12; ++i) v.c[i] = conj(c) * v.c[i];
    store_spinor<P>(out.base + rhs * out.rs, cb, out.n, v);
}

hipError_t launch_twist_apply(const Geom &g, double c_re, double c_im, FieldView out, FieldView in, hipStream_t s)
{
    const dim3 grid((g.vh + 255) / 256, in.nrhs);
    switch (in.prec) {
    case F64: twist_apply_kernel<F64><<<grid, 256, 0, s>>>(g, c_re, c_im, out, in); break;
    case F32: twist_apply_kernel<F32><<<grid, 256, 0, s>>>(g, c_re, c_im, out, in); break;
    case F16: twist_apply_kernel<F16><<<grid, 256, 0, s>>>(g, c_re, c_im, out, in); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_clover_build(const Geom &g, const char *links64, double csw, double kappa, int traceless,
                               char *fbuf, char *clov64, hipStream_t s)
{
    field_strength_kernel<<<dim3((g.vh + 127) / 128, 6, 2), 128, 0, s>>>(g, links64, traceless, fbuf);
    clover_build_kernel<<<dim3((g.vh + 127) / 128, 2), 128, 0, s>>>(g, fbuf, csw, kappa, clov64);
    return hipGetLastError();
}

hipError_t launch_clover_invert(const Geom &g, int p, const char *clov64, char *inv64, int *flag, hipStream_t s)
{
    clover_invert_kernel<<<dim3((2 * g.vh + INV_T - 1) / INV_T), INV_T, 0, s>>>(g, p, clov64, inv64, flag);
    return hipGetLastError();
}

hipError_t launch_convert_clover(const Geom &g, const char *clov64, int prec, char *dst, hipStream_t s, int p0, int np)
{
    if (p0 < 0 || np < 1 || p0 + np > 2) return hipErrorInvalidValue;
    const dim3 grid((g.vh + 255) / 256, np);
    if (prec == F32) convert_clover_kernel<F32><<<grid, 256, 0, s>>>(g, p0, clov64, dst);
    else if (prec == F16) convert_clover_kernel<F16><<<grid, 256, 0, s>>>(g, p0, clov64, dst);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_clover_apply(const Geom &g, const char *clov, FieldView out, FieldView in, hipStream_t s)
{
    const dim3 grid((g.vh + 255) / 256, in.nrhs);
    switch (in.prec) {
    case F64: clover_apply_kernel<F64><<<grid, 256, 0, s>>>(g, clov, out, in); break;
    case F32: clover_apply_kernel<F32><<<grid, 256, 0, s>>>(g, clov, out, in); break;
    case F16: clover_apply_kernel<F16><<<grid, 256, 0, s>>>(g, clov, out, in); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lq
