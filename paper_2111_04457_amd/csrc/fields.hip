// fields.hip -- field import/export, link packing and the clover term.
#include "fields.h"
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

struct M3 {
    cx<double> e[9];
};

__device__ __forceinline__ M3 link_at(const Geom &g, const char *links64, const int c[4], int mu)
{
    const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
    M3 m;
    double raw[18];
    load_planes<double, 18>(links64 + (long)(p * 4 + mu) * link_bytes(F64, 18, g.vh), cb_index(g, c), g.vh, raw);
#pragma unroll
    for (int i = 0; i < 9; ++i) m.e[i] = cx<double>{raw[2 * i], raw[2 * i + 1]};
    return m;
}

__device__ __forceinline__ M3 mul(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c.e[i * 3 + j] = a.e[i * 3 + 0] * b.e[0 * 3 + j] + a.e[i * 3 + 1] * b.e[1 * 3 + j] +
                             a.e[i * 3 + 2] * b.e[2 * 3 + j];
    return c;
}

__device__ __forceinline__ M3 dag(const M3 &a)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.e[i * 3 + j] = conj(a.e[j * 3 + i]);
    return c;
}

__device__ __forceinline__ void shift(const Geom &g, const int c[4], int mu, int dm, int nu, int dn, int o[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = c[k];
    o[mu] = (o[mu] + dm + g.L[mu]) % g.L[mu];
    o[nu] = (o[nu] + dn + g.L[nu]) % g.L[nu];
}

// Fhat_{mu nu}(x) = (Q - Q^dag)/8 from the four counter-clockwise leaves;
// colour trace removed if traceless.
__device__ M3 field_strength(const Geom &g, const char *links64, const int c[4], int mu, int nu, int traceless)
{
    int s1[4], s2[4], s3[4];
    M3 Q, t;
    // leaf in the (+mu, +nu) quadrant
    shift(g, c, mu, 1, nu, 0, s1);
    shift(g, c, mu, 0, nu, 1, s2);
    Q = mul(mul(link_at(g, links64, c, mu), link_at(g, links64, s1, nu)),
            mul(dag(link_at(g, links64, s2, mu)), dag(link_at(g, links64, c, nu))));
    // (-mu, +nu) quadrant: x -> x+nu -> x+nu-mu -> x-mu -> x
    shift(g, c, mu, -1, nu, 1, s1);
    shift(g, c, mu, -1, nu, 0, s2);
    t = mul(mul(link_at(g, links64, c, nu), dag(link_at(g, links64, s1, mu))),
            mul(dag(link_at(g, links64, s2, nu)), link_at(g, links64, s2, mu)));
#pragma unroll
    for (int i = 0; i < 9; ++i) Q.e[i] = Q.e[i] + t.e[i];
    // (-mu, -nu) quadrant: x -> x-mu -> x-mu-nu -> x-nu -> x
    shift(g, c, mu, -1, nu, -1, s1);
    shift(g, c, mu, 0, nu, -1, s3);
    t = mul(mul(dag(link_at(g, links64, s2, mu)), dag(link_at(g, links64, s1, nu))),
            mul(link_at(g, links64, s1, mu), link_at(g, links64, s3, nu)));
#pragma unroll
    for (int i = 0; i < 9; ++i) Q.e[i] = Q.e[i] + t.e[i];
    // (+mu, -nu) quadrant: x -> x-nu -> x-nu+mu -> x+mu -> x
    shift(g, c, mu, 1, nu, -1, s1);
    t = mul(mul(dag(link_at(g, links64, s3, nu)), link_at(g, links64, s3, mu)),
            mul(link_at(g, links64, s1, nu), dag(link_at(g, links64, c, mu))));
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
// and the clover block is A = 1 - c_sw kappa times it.
__global__ __launch_bounds__(128) void clover_build_kernel(Geom g, const char *links64, double csw, double kappa,
                                                          int traceless, char *clov64)
{
    const int cb = blockIdx.x * 128 + threadIdx.x;
    const int p = blockIdx.y;
    if (cb >= g.vh) return;
    int c[4];
    cb_coords(g, p, cb, c);
    const M3 Fxy = field_strength(g, links64, c, 0, 1, traceless);
    const M3 Fxz = field_strength(g, links64, c, 0, 2, traceless);
    const M3 Fyz = field_strength(g, links64, c, 1, 2, traceless);
    const M3 Fxt = field_strength(g, links64, c, 0, 3, traceless);
    const M3 Fyt = field_strength(g, links64, c, 1, 3, traceless);
    const M3 Fzt = field_strength(g, links64, c, 2, 3, traceless);
    double out[72];
    const double ck = -csw * kappa;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const double eta = b == 0 ? -1.0 : 1.0;
        cx<double> X[9], Y[9], Z[9], blk[6][6];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            X[i] = Fyz.e[i] + eta * Fxt.e[i];
            Y[i] = Fxz.e[i] - eta * Fyt.e[i];
            Z[i] = Fxy.e[i] + eta * Fzt.e[i];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int k = a * 3 + d;
                blk[a][d] = ck * ti(Z[k]);
                blk[a][3 + d] = ck * (ti(X[k]) - Y[k]);
                blk[3 + a][d] = ck * (ti(X[k]) + Y[k]);
                blk[3 + a][3 + d] = ck * tmi(Z[k]);
            }
        double *o = out + 36 * b;
#pragma unroll
        for (int i = 0; i < 6; ++i) o[i] = 1.0 + blk[i][i].re;
        int k = 6;
#pragma unroll
        for (int i = 1; i < 6; ++i)
#pragma unroll
            for (int j = 0; j < i; ++j) {
                o[k++] = blk[i][j].re;
                o[k++] = blk[i][j].im;
            }
    }
    store_planes<double, 72>(clov64 + (long)p * clover_bytes(F64, g.vh), cb, g.vh, out);
}

// One 6x6 Hermitian block per thread: unpack, Gauss-Jordan with partial
// pivoting on [A | 1], pack the lower triangle of the inverse.
__global__ __launch_bounds__(64) void clover_invert_kernel(Geom g, const char *clov64, char *inv64,
                                                          int *flag)
{
    const int idx = blockIdx.x * 64 + threadIdx.x;
    const int p = blockIdx.y;
    if (idx >= 2 * g.vh) return;
    const int cb = idx >> 1, b = idx & 1;
    const char *base = clov64 + (long)p * clover_bytes(F64, g.vh);
    double raw[72];
    load_planes<double, 72>(base, cb, g.vh, raw);
    const double *c = raw + 36 * b;
    cx<double> a[6][12];
    double scale = 0.0;
    for (int i = 0; i < 6; ++i) {
        a[i][i] = cx<double>{c[i], 0.0};
        for (int j = 0; j < 6; ++j) a[i][6 + j] = cx<double>{i == j ? 1.0 : 0.0, 0.0};
    }
    int k = 6;
    for (int i = 1; i < 6; ++i)
        for (int j = 0; j < i; ++j) {
            a[i][j] = cx<double>{c[k], c[k + 1]};
            a[j][i] = cx<double>{c[k], -c[k + 1]};
            k += 2;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) scale = fmax(scale, sqrt(norm2(a[i][j])));
    bool sing = false;
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        double best = norm2(a[col][col]);
        for (int r = col + 1; r < 6; ++r) {
            const double v = norm2(a[r][col]);
            if (v > best) { best = v; piv = r; }
        }
        if (!(sqrt(best) > 1e-14 * scale)) { sing = true; break; }
        if (piv != col)
            for (int j = 0; j < 12; ++j) {
                const cx<double> t = a[col][j];
                a[col][j] = a[piv][j];
                a[piv][j] = t;
            }
        const double d = norm2(a[col][col]);
        const cx<double> inv = cx<double>{a[col][col].re / d, -a[col][col].im / d};
        for (int j = 0; j < 12; ++j) a[col][j] = inv * a[col][j];
        for (int r = 0; r < 6; ++r) {
            if (r == col) continue;
            const cx<double> f = a[r][col];
            for (int j = 0; j < 12; ++j) a[r][j] = a[r][j] - f * a[col][j];
        }
    }
    if (sing) atomicOr(flag, 1);
    // write this block's 36 reals into a local copy of the site record;
    // the two blocks of a site are owned by neighbouring threads, so each
    // writes only its own half of every plane element.
    double o[36];
    for (int i = 0; i < 6; ++i) o[i] = sing ? 0.0 : a[i][6 + i].re;
    k = 6;
    for (int i = 1; i < 6; ++i)
        for (int j = 0; j < i; ++j) {
            // Hermitian average of the (i, j) and conj (j, i) entries
            o[k++] = sing ? 0.0 : 0.5 * (a[i][6 + j].re + a[j][6 + i].re);
            o[k++] = sing ? 0.0 : 0.5 * (a[i][6 + j].im - a[j][6 + i].im);
        }
    char *dst = inv64 + (long)p * clover_bytes(F64, g.vh);
    // 72 FP64 reals = 36 planes of 16 bytes; block b owns planes 18b..18b+17
    for (int q = 0; q < 18; ++q) {
        double2 v;
        v.x = o[2 * q];
        v.y = o[2 * q + 1];
        *reinterpret_cast<double2 *>(dst + ((long)(18 * b + q) * g.vh + cb) * 16) = v;
    }
}

template <int P>
__global__ __launch_bounds__(256) void convert_clover_kernel(Geom g, const char *clov64, char *dst)
{
    using S = typename PT<P>::S;
    const int cb = blockIdx.x * 256 + threadIdx.x;
    const int p = blockIdx.y;
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

hipError_t launch_clover_build(const Geom &g, const char *links64, double csw, double kappa, int traceless,
                               char *clov64, hipStream_t s)
{
    clover_build_kernel<<<dim3((g.vh + 127) / 128, 2), 128, 0, s>>>(g, links64, csw, kappa, traceless, clov64);
    return hipGetLastError();
}

hipError_t launch_clover_invert(const Geom &g, const char *clov64, char *inv64, int *flag, hipStream_t s)
{
    clover_invert_kernel<<<dim3((2 * g.vh + 63) / 64, 2), 64, 0, s>>>(g, clov64, inv64, flag);
    return hipGetLastError();
}

hipError_t launch_convert_clover(const Geom &g, const char *clov64, int prec, char *dst, hipStream_t s)
{
    const dim3 grid((g.vh + 255) / 256, 2);
    if (prec == F32) convert_clover_kernel<F32><<<grid, 256, 0, s>>>(g, clov64, dst);
    else if (prec == F16) convert_clover_kernel<F16><<<grid, 256, 0, s>>>(g, clov64, dst);
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
