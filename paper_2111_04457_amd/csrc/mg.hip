// mg.hip -- two-level adaptive-aggregation multigrid for D x = b.
//
// Sec. 1 cites adaptive multigrid as the solver of choice near the physical
// quark masses and Sec. 4 lists multigrid among the solver algorithms,
// without details; this is the adaptive-aggregation reading: a prolongator P
// built from near-null vectors split by chirality and orthonormalised per
// aggregate, the Galerkin coarse operator D_c = P^dag D P as a 9-point
// stencil of dense blocks, and a cycle (coarse correction, then a
// minimal-residual smoother) preconditioning flexible GCR inside the FP64
// defect correction.
//
// Device layout: the near-null vectors are nvec FP32 full packed fields
// ([vector][parity][planes]); a coarse vector is an FP32 field of
// "pseudo-sites" holding 12 complex numbers each (element e = A * 2 nvec + r
// at pseudo-site e / 12, component e % 12), so the solver's vector kernels
// and its device-resident BiCGStab run on it unchanged; the coarse operator
// is FP32 complex [aggregate][9][2 nvec][2 nvec].
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "solver.h"

namespace lq {

struct MgGeom {
    Geom g;
    int bl[4];     // aggregate extents
    int lc[4];     // coarse extents
    int nagg;      // coarse sites
    int asz;       // sites per aggregate
    int nv;        // near-null vectors
    int n2;        // coarse dof per aggregate (2 nv)
    long vstride;  // bytes between two of the FP32 full fields of the vectors
};

namespace {

constexpr int MT = 256;  // threads per workgroup
constexpr int BC = 8;    // aggregate sites staged per step of the coarse-operator build
constexpr int PMAX = 4;  // (row, column) pairs per thread of the build: 64 x 16 / 256

__device__ __forceinline__ void agg_coords(const MgGeom &m, int A, int a[4])
{
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        a[mu] = A % m.lc[mu];
        A /= m.lc[mu];
    }
}

__device__ __forceinline__ int agg_index(const MgGeom &m, const int a[4])
{
    return a[0] + m.lc[0] * (a[1] + m.lc[1] * (a[2] + m.lc[2] * a[3]));
}

__device__ __forceinline__ int color_of(const int a[4])
{
    return (a[0] & 1) | ((a[1] & 1) << 1) | ((a[2] & 1) << 2) | ((a[3] & 1) << 3);
}

// coordinates of site l (lexicographic in the block, x fastest) of aggregate a
__device__ __forceinline__ void agg_site(const MgGeom &m, const int a[4], int l, int c[4])
{
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = a[mu] * m.bl[mu] + l % m.bl[mu];
        l /= m.bl[mu];
    }
}

__device__ __forceinline__ int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

// element e of a coarse pseudo-site field (FP32 packed, 12 complex per pseudo-site)
__device__ __forceinline__ float2 *celem(char *base, long e)
{
    const long s = e / 12;
    const int f = 2 * (int)(e % 12);  // float index of the real part in the 24-float record
    return reinterpret_cast<float2 *>(base + (s >> 6) * (96L * SB) + (long)(f >> 2) * (16 * SB) + (s & 63) * 16 +
                                      (f & 3) * 4);
}
__device__ __forceinline__ float2 cget(const char *base, long e) { return *celem(const_cast<char *>(base), e); }

__device__ __forceinline__ const char *vec_site(const MgGeom &m, const char *V, int k, int p)
{
    return V + (long)k * m.vstride + (long)p * spinor_field_bytes(F32, m.g.vh);
}

// Per aggregate and chirality, modified Gram-Schmidt of the vectors' halves
// in vector order (FP64 sums, FP32 storage); a vanishing half stays zero.
__global__ __launch_bounds__(MT) void mg_orth_kernel(MgGeom m, char *V)
{
    int a[4];
    agg_coords(m, blockIdx.x, a);
    __shared__ double lds[MT / 64];
    __shared__ double bc[2];
    for (int chi = 0; chi < 2; ++chi) {
        const int c0 = 6 * chi;
        for (int k = 0; k < m.nv; ++k) {
            for (int j = 0; j <= k; ++j) {
                double re = 0, im = 0;
                for (int l = threadIdx.x; l < m.asz; l += MT) {
                    int c[4];
                    agg_site(m, a, l, c);
                    const int p = parity_of(c), cb = cb_index(m.g, c);
                    const Spinor<float> x = load_spinor<F32>(vec_site(m, V, k, p), cb, m.g.vh);
                    const Spinor<float> y = load_spinor<F32>(vec_site(m, V, j, p), cb, m.g.vh);
#pragma unroll
                    for (int i = 0; i < 6; ++i) {
                        const cx<float> u = y.c[c0 + i], v = x.c[c0 + i];
                        re += (double)u.re * v.re + (double)u.im * v.im;
                        im += (double)u.re * v.im - (double)u.im * v.re;
                    }
                }
                re = block_sum<MT>(re, lds);
                im = block_sum<MT>(im, lds);
                if (threadIdx.x == 0) {
                    bc[0] = re;
                    bc[1] = im;
                }
                __syncthreads();
                re = bc[0];
                im = bc[1];
                __syncthreads();
                // j < k: x -= <y, x> y; j == k: x /= |x| (re = |x|^2)
                const float fr = j < k ? (float)re : (re > 0 ? (float)(1.0 / sqrt(re)) : 0.0f);
                const float fi = j < k ? (float)im : 0.0f;
                for (int l = threadIdx.x; l < m.asz; l += MT) {
                    int c[4];
                    agg_site(m, a, l, c);
                    const int p = parity_of(c), cb = cb_index(m.g, c);
                    char *xb = const_cast<char *>(vec_site(m, V, k, p));
                    Spinor<float> x = load_spinor<F32>(xb, cb, m.g.vh);
                    if (j < k) {
                        const Spinor<float> y = load_spinor<F32>(vec_site(m, V, j, p), cb, m.g.vh);
#pragma unroll
                        for (int i = 0; i < 6; ++i) {
                            const cx<float> u = y.c[c0 + i];
                            x.c[c0 + i].re -= fr * u.re - fi * u.im;
                            x.c[c0 + i].im -= fr * u.im + fi * u.re;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 6; ++i) {
                            x.c[c0 + i].re *= fr;
                            x.c[c0 + i].im *= fr;
                        }
                    }
                    store_spinor<F32>(xb, cb, m.g.vh, x);
                }
            }
        }
    }
}

// coarse[A][chi * nv + k] = sum over A's sites of v_k(x)_chi^dag f(x)_chi
// (f an FP32 full packed field): one pass over the aggregate's sites per 8
// vectors, each site's f loaded once; per-wavefront sums, then the waves in
// order.
__global__ __launch_bounds__(MT) void mg_restrict_kernel(MgGeom m, const char *V, const char *f, char *coarse)
{
    const int A = blockIdx.x;
    int a[4];
    agg_coords(m, A, a);
    __shared__ double red[MT / 64][2][16];
    const long fbytes = spinor_field_bytes(F32, m.g.vh);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k0 = 0; k0 < m.nv; k0 += 8) {
        double re[16], im[16];  // index chi * 8 + q for vector k0 + q
#pragma unroll
        for (int i = 0; i < 16; ++i) re[i] = im[i] = 0.0;
        for (int l = threadIdx.x; l < m.asz; l += MT) {
            int c[4];
            agg_site(m, a, l, c);
            const int p = parity_of(c), cb = cb_index(m.g, c);
            const Spinor<float> x = load_spinor<F32>(f + p * fbytes, cb, m.g.vh);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (k0 + q >= m.nv) break;
                const Spinor<float> v = load_spinor<F32>(vec_site(m, V, k0 + q, p), cb, m.g.vh);
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    const cx<float> u = v.c[i], w = x.c[i];
                    const int slot = (i / 6) * 8 + q;
                    re[slot] += (double)u.re * w.re + (double)u.im * w.im;
                    im[slot] += (double)u.re * w.im - (double)u.im * w.re;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const double sr = wave_sum(re[i]), si = wave_sum(im[i]);
            if (lane == 0) {
                red[wv][0][i] = sr;
                red[wv][1][i] = si;
            }
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            const int i = threadIdx.x, chi = i / 8, k = k0 + i % 8;
            if (k < m.nv) {
                double sr = 0, si = 0;
                for (int w = 0; w < MT / 64; ++w) {
                    sr += red[w][0][i];
                    si += red[w][1][i];
                }
                *celem(coarse, (long)A * m.n2 + chi * m.nv + k) = make_float2((float)sr, (float)si);
            }
        }
        __syncthreads();
    }
}

// f(x) = sum_k v_k(x)_chi coarse[A(x)][chi * nv + k] over both chiralities
__global__ __launch_bounds__(MT) void mg_prolong_kernel(MgGeom m, const char *V, const char *coarse, char *f)
{
    const int cb = blockIdx.x * MT + threadIdx.x;
    const int p = blockIdx.y;
    if (cb >= m.g.vh) return;
    int c[4], a[4];
    cb_coords(m.g, p, cb, c);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) a[mu] = c[mu] / m.bl[mu];
    const long e0 = (long)agg_index(m, a) * m.n2;
    Spinor<float> out;
#pragma unroll
    for (int i = 0; i < 12; ++i) out.c[i] = cx<float>{0.0f, 0.0f};
    for (int k = 0; k < m.nv; ++k) {
        const Spinor<float> v = load_spinor<F32>(vec_site(m, V, k, p), cb, m.g.vh);
        const float2 u = cget(coarse, e0 + k), w = cget(coarse, e0 + m.nv + k);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            out.c[i].re += v.c[i].re * u.x - v.c[i].im * u.y;
            out.c[i].im += v.c[i].re * u.y + v.c[i].im * u.x;
            out.c[6 + i].re += v.c[6 + i].re * w.x - v.c[6 + i].im * w.y;
            out.c[6 + i].im += v.c[6 + i].re * w.y + v.c[6 + i].im * w.x;
        }
    }
    store_spinor<F32>(f + (long)p * spinor_field_bytes(F32, m.g.vh), cb, m.g.vh, out);
}

// y[A][r] = sum_d sum_c Dc[A][d][r][c] x[nbr(A, d)][c]; nothing if the
// system is frozen (mask: its solver scalars).  One workgroup per
// aggregate: the nine neighbours' coarse vectors in LDS, one thread per
// (d, r) row product (rows contiguous in memory across the threads), then
// the sum over d in order.
__global__ __launch_bounds__(MT) void mg_capply_kernel(MgGeom m, const float2 *__restrict__ Dc, const char *x,
                                                      char *y, const double *mask)
{
    if (mask && (mask[SC_DONE] != 0.0 || mask[SC_BREAK] != 0.0)) return;
    __shared__ float2 xs[9][64];
    __shared__ float2 part[9][64];
    const int A = blockIdx.x, n2 = m.n2;
    int a[4];
    agg_coords(m, A, a);
    for (int q = threadIdx.x; q < 9 * n2; q += MT) {
        const int d = q / n2, c = q % n2;
        int b[4] = {a[0], a[1], a[2], a[3]};
        if (d > 0) {
            const int mu = (d - 1) >> 1;
            b[mu] = (d & 1) ? (b[mu] + 1) % m.lc[mu] : (b[mu] + m.lc[mu] - 1) % m.lc[mu];
        }
        xs[d][c] = cget(x, (long)agg_index(m, b) * n2 + c);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 9 * n2; q += MT) {
        const int d = q / n2, r = q % n2;
        const float2 *row = Dc + (((long)A * 9 + d) * n2 + r) * n2;
        float ar = 0.0f, ai = 0.0f;
        for (int c = 0; c < n2; ++c) {
            const float2 u = row[c], v = xs[d][c];
            ar = __builtin_fmaf(u.x, v.x, ar);
            ar = __builtin_fmaf(-u.y, v.y, ar);
            ai = __builtin_fmaf(u.x, v.y, ai);
            ai = __builtin_fmaf(u.y, v.x, ai);
        }
        part[d][r] = make_float2(ar, ai);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n2; r += MT) {
        float sr = 0.0f, si = 0.0f;
        for (int d = 0; d < 9; ++d) {
            sr += part[d][r].x;
            si += part[d][r].y;
        }
        *celem(y, (long)A * n2 + r) = make_float2(sr, si);
    }
}

// Z_j (FP64 full fields): column col0 + j of P (chirality half chi of v_k,
// col = chi * nv + k) on the aggregates of the given colour, zero elsewhere
__global__ __launch_bounds__(MT) void mg_column_kernel(MgGeom m, const char *V, int color, int col0, int ncol, char *Z,
                                                      long zstride)
{
    const int cb = blockIdx.x * MT + threadIdx.x;
    const int p = blockIdx.y;
    if (cb >= m.g.vh) return;
    int c[4], a[4];
    cb_coords(m.g, p, cb, c);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) a[mu] = c[mu] / m.bl[mu];
    const bool on = color_of(a) == color;
    const long f64 = spinor_field_bytes(F64, m.g.vh);
    for (int j = 0; j < ncol; ++j) {
        const int col = col0 + j, chi = col / m.nv, k = col % m.nv;
        Spinor<double> z;
#pragma unroll
        for (int i = 0; i < 12; ++i) z.c[i] = cx<double>{0.0, 0.0};
        if (on) {
            const Spinor<float> v = load_spinor<F32>(vec_site(m, V, k, p), cb, m.g.vh);
#pragma unroll
            for (int i = 0; i < 6; ++i) z.c[6 * chi + i] = cx<double>{v.c[6 * chi + i].re, v.c[6 * chi + i].im};
        }
        store_spinor<F64>(Z + j * zstride + p * f64, cb, m.g.vh, z);
    }
}

// Entries Dc[A][d][r][col0 + j] = sum over the sites x of A whose
// contributions in W_j = D Z_j come from the aggregate of the given colour
// (A itself: d = 0; the aggregate at +mu or -mu, when the colours differ in
// bit mu only: the sites on A's +mu face give d = 1 + 2 mu, those on the
// -mu face d = 2 + 2 mu) of v_k(x)_chi^dag W_j(x)_chi, r = chi * nv + k.
// Every entry is written by exactly one (colour, column) launch.
__global__ __launch_bounds__(MT) void mg_build_kernel(MgGeom m, const char *V, const char *W, long wstride, int color,
                                                     int col0, int ncol, float2 *Dc)
{
    extern __shared__ float2 sm[];
    float2 *Vs = sm;                      // [nv][BC][12]
    float2 *Ws = sm + m.nv * BC * 12;     // [ncol][BC][12]
    int *cls = reinterpret_cast<int *>(Ws + ncol * BC * 12);  // [BC]: -1 none, 0 self or +mu, 1 -mu
    const int A = blockIdx.x;
    int a[4];
    agg_coords(m, A, a);
    const int diff = color_of(a) ^ color;
    if (diff & (diff - 1)) return;  // two or more colour bits differ: no contribution
    const int mu = diff ? __builtin_ctz(diff) : -1;
    const int npair = m.n2 * ncol;
    float2 acc0[PMAX], acc1[PMAX];
#pragma unroll
    for (int q = 0; q < PMAX; ++q) acc0[q] = acc1[q] = make_float2(0.0f, 0.0f);
    const long f32 = spinor_field_bytes(F32, m.g.vh), f64 = spinor_field_bytes(F64, m.g.vh);
    for (int s0 = 0; s0 < m.asz; s0 += BC) {
        __syncthreads();
        for (int q = threadIdx.x; q < (m.nv + ncol) * BC; q += MT) {
            const int vec = q / BC, si = q % BC, l = s0 + si;
            if (l >= m.asz) {
                if (vec == 0) cls[si] = -1;
                continue;
            }
            int c[4];
            agg_site(m, a, l, c);
            const int p = parity_of(c), cb = cb_index(m.g, c);
            if (vec < m.nv) {
                const Spinor<float> v = load_spinor<F32>(V + (long)vec * m.vstride + p * f32, cb, m.g.vh);
#pragma unroll
                for (int i = 0; i < 12; ++i) Vs[(vec * BC + si) * 12 + i] = make_float2(v.c[i].re, v.c[i].im);
            } else {
                const Spinor<double> w = load_spinor<F64>(W + (long)(vec - m.nv) * wstride + p * f64, cb, m.g.vh);
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    Ws[((vec - m.nv) * BC + si) * 12 + i] = make_float2((float)w.c[i].re, (float)w.c[i].im);
            }
            if (vec == 0) {
                int k = 0;
                if (mu >= 0) {
                    const int pos = c[mu] % m.bl[mu];
                    k = pos == m.bl[mu] - 1 ? 0 : pos == 0 ? 1 : -1;
                }
                cls[si] = k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PMAX; ++q) {
            const int pair = threadIdx.x + q * MT;
            if (pair >= npair) break;
            const int r = pair / ncol, j = pair % ncol, chi = r / m.nv, k = r % m.nv;
            for (int si = 0; si < BC; ++si) {
                const int cl = cls[si];
                if (cl < 0) continue;
                const float2 *v = Vs + (k * BC + si) * 12 + 6 * chi;
                const float2 *w = Ws + (j * BC + si) * 12 + 6 * chi;
                float dr = 0.0f, di = 0.0f;
#pragma unroll
                for (int i = 0; i < 6; ++i) {
                    dr = __builtin_fmaf(v[i].x, w[i].x, dr);
                    dr = __builtin_fmaf(v[i].y, w[i].y, dr);
                    di = __builtin_fmaf(v[i].x, w[i].y, di);
                    di = __builtin_fmaf(-v[i].y, w[i].x, di);
                }
                if (cl == 0) {
                    acc0[q].x += dr;
                    acc0[q].y += di;
                } else {
                    acc1[q].x += dr;
                    acc1[q].y += di;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
        const int pair = threadIdx.x + q * MT;
        if (pair >= npair) break;
        const int r = pair / ncol, col = col0 + pair % ncol;
        const int d0 = mu < 0 ? 0 : 1 + 2 * mu;
        Dc[(((long)A * 9 + d0) * m.n2 + r) * m.n2 + col] = acc0[q];
        if (mu >= 0) Dc[(((long)A * 9 + 2 + 2 * mu) * m.n2 + r) * m.n2 + col] = acc1[q];
    }
}

// ---------------------------------------------------- fine-level vector kernels
// (FP32 full fields: two slices of vh sites, rs bytes apart)

__device__ __forceinline__ char *slice_of(const FieldView &v, int sl) { return v.base + (long)sl * v.rs; }

// partial[((j * 2) + slice) * nb + blk] = (re, im) of <X_j, x> over the block
__global__ __launch_bounds__(MT) void mg_mdot_kernel(const char *X, long xstride, int nx, FieldView x,
                                                    double *partial)
{
    const int nb = gridDim.x, sl = blockIdx.y, j0 = blockIdx.z * 8;
    const long i = (long)blockIdx.x * MT + threadIdx.x;
    double re[8], im[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) re[q] = im[q] = 0.0;
    if (i < x.n) {
        const Spinor<float> xv = load_spinor<F32>(slice_of(x, sl), i, x.n);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (j0 + q >= nx) break;
            const Spinor<float> u = load_spinor<F32>(X + (long)(j0 + q) * xstride + (long)sl * x.rs, i, x.n);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                re[q] += (double)u.c[c].re * xv.c[c].re + (double)u.c[c].im * xv.c[c].im;
                im[q] += (double)u.c[c].re * xv.c[c].im - (double)u.c[c].im * xv.c[c].re;
            }
        }
    }
    __shared__ double lds[MT / 64];
    for (int q = 0; q < 8; ++q) {
        if (j0 + q >= nx) break;
        const double a = block_sum<MT>(re[q], lds);
        const double b = block_sum<MT>(im[q], lds);
        if (threadIdx.x == 0) {
            double *o = partial + (((long)(j0 + q) * 2 + sl) * nb + blockIdx.x) * 2;
            o[0] = a;
            o[1] = b;
        }
    }
}

// y -= sum_j coef_j X_j (coef: device complex, FP64)
__global__ __launch_bounds__(MT) void mg_maxpy_kernel(FieldView y, const char *X, long xstride, int nx,
                                                     const double *coef)
{
    const int sl = blockIdx.y;
    const long i = (long)blockIdx.x * MT + threadIdx.x;
    if (i >= y.n) return;
    Spinor<float> yv = load_spinor<F32>(slice_of(y, sl), i, y.n);
    for (int j = 0; j < nx; ++j) {
        const Spinor<float> u = load_spinor<F32>(X + (long)j * xstride + (long)sl * y.rs, i, y.n);
        const float cr = (float)coef[2 * j], ci = (float)coef[2 * j + 1];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            yv.c[c].re -= cr * u.c[c].re - ci * u.c[c].im;
            yv.c[c].im -= cr * u.c[c].im + ci * u.c[c].re;
        }
    }
    store_spinor<F32>(slice_of(y, sl), i, y.n, yv);
}

// e += alpha z, r -= alpha w, partial |r|^2 per (slice, block)
__global__ __launch_bounds__(MT) void mg_gcr_update_kernel(FieldView e, FieldView z, FieldView r, FieldView w,
                                                          double ar_, double ai_, double *partial)
{
    const int sl = blockIdx.y;
    const long i = (long)blockIdx.x * MT + threadIdx.x;
    double s = 0.0;
    if (i < e.n) {
        const float ar = (float)ar_, ai = (float)ai_;
        Spinor<float> ev = load_spinor<F32>(slice_of(e, sl), i, e.n);
        Spinor<float> rv = load_spinor<F32>(slice_of(r, sl), i, r.n);
        const Spinor<float> zv = load_spinor<F32>(slice_of(z, sl), i, z.n);
        const Spinor<float> wv = load_spinor<F32>(slice_of(w, sl), i, w.n);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            ev.c[c].re += ar * zv.c[c].re - ai * zv.c[c].im;
            ev.c[c].im += ar * zv.c[c].im + ai * zv.c[c].re;
            rv.c[c].re -= ar * wv.c[c].re - ai * wv.c[c].im;
            rv.c[c].im -= ar * wv.c[c].im + ai * wv.c[c].re;
            s += (double)rv.c[c].re * rv.c[c].re + (double)rv.c[c].im * rv.c[c].im;
        }
        store_spinor<F32>(slice_of(e, sl), i, e.n, ev);
        store_spinor<F32>(slice_of(r, sl), i, r.n, rv);
    }
    __shared__ double lds[MT / 64];
    const double t = block_sum<MT>(s, lds);
    if (threadIdx.x == 0) partial[(long)sl * gridDim.x + blockIdx.x] = t;
}

// s = r - t; d = 0
__global__ __launch_bounds__(MT) void mg_smooth_init_kernel(FieldView s, FieldView r, FieldView t, FieldView d)
{
    const int sl = blockIdx.y;
    const long i = (long)blockIdx.x * MT + threadIdx.x;
    if (i >= s.n) return;
    const Spinor<float> rv = load_spinor<F32>(slice_of(r, sl), i, r.n);
    const Spinor<float> tv = load_spinor<F32>(slice_of(t, sl), i, t.n);
    Spinor<float> o, z;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        o.c[c] = cx<float>{rv.c[c].re - tv.c[c].re, rv.c[c].im - tv.c[c].im};
        z.c[c] = cx<float>{0.0f, 0.0f};
    }
    store_spinor<F32>(slice_of(s, sl), i, s.n, o);
    store_spinor<F32>(slice_of(d, sl), i, d.n, z);
}

// minimal-residual step: d += omega s, s -= omega q (omega from the scalars)
__global__ __launch_bounds__(MT) void mg_mr_kernel(FieldView d, FieldView s, FieldView q, const double *sc)
{
    const int sl = blockIdx.y;
    const long i = (long)blockIdx.x * MT + threadIdx.x;
    if (i >= d.n) return;
    const float wr = (float)sc[SC_OMEGA_RE], wi = (float)sc[SC_OMEGA_IM];
    Spinor<float> dv = load_spinor<F32>(slice_of(d, sl), i, d.n);
    Spinor<float> sv = load_spinor<F32>(slice_of(s, sl), i, s.n);
    const Spinor<float> qv = load_spinor<F32>(slice_of(q, sl), i, q.n);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        dv.c[c].re += wr * sv.c[c].re - wi * sv.c[c].im;
        dv.c[c].im += wr * sv.c[c].im + wi * sv.c[c].re;
        sv.c[c].re -= wr * qv.c[c].re - wi * qv.c[c].im;
        sv.c[c].im -= wr * qv.c[c].im + wi * qv.c[c].re;
    }
    store_spinor<F32>(slice_of(d, sl), i, d.n, dv);
    store_spinor<F32>(slice_of(s, sl), i, s.n, sv);
}

// z += d
__global__ __launch_bounds__(MT) void mg_add_kernel(FieldView z, FieldView d)
{
    const int sl = blockIdx.y;
    const long i = (long)blockIdx.x * MT + threadIdx.x;
    if (i >= z.n) return;
    Spinor<float> zv = load_spinor<F32>(slice_of(z, sl), i, z.n);
    const Spinor<float> dv = load_spinor<F32>(slice_of(d, sl), i, d.n);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        zv.c[c].re += dv.c[c].re;
        zv.c[c].im += dv.c[c].im;
    }
    store_spinor<F32>(slice_of(z, sl), i, z.n, zv);
}

// coarse pseudo-site field <-> complex128 [ncoarse][n2]
__global__ __launch_bounds__(MT) void mg_cimport_kernel(long n, const double *src, char *dst)
{
    const long e = (long)blockIdx.x * MT + threadIdx.x;
    if (e < n) *celem(dst, e) = make_float2((float)src[2 * e], (float)src[2 * e + 1]);
}
__global__ __launch_bounds__(MT) void mg_cexport_kernel(long n, const char *src, double *dst)
{
    const long e = (long)blockIdx.x * MT + threadIdx.x;
    if (e < n) {
        const float2 v = cget(src, e);
        dst[2 * e] = v.x;
        dst[2 * e + 1] = v.y;
    }
}

}  // namespace

}  // namespace lq

using namespace lq;

struct lq_mg {
    lq_op *op = nullptr;
    lq_mg_params prm{};
    MgGeom m{};
    long npseudo = 0;          // pseudo-sites of a coarse vector
    long cbytes = 0;           // bytes of one coarse vector
    Buf vecs;                  // nv FP32 full fields
    Buf dc;                    // coarse operator
    Buf cws;                   // 10 coarse vectors: the coarse BiCGStab's nine, and its source
    Buf csc, cpart;            // coarse solver scalars and partial sums
    double *chsc = nullptr;    // pinned mirror of the coarse scalars
    Buf fws;                   // FP32 full fields: z[m], w[m], r, e, s, q, d, t
    Buf f64ws;                 // FP64 full fields: b, x, r, t
    Buf part;                  // partial sums of the fine-level reductions
    Buf coef;                  // device coefficients of mg_maxpy_kernel
    Buf osc;                   // scalars: [0] outer residual, [1] smoother
    double *ohsc = nullptr;    // pinned mirror
    std::vector<double> hpart;  // host copy of partials
    long id = 0;               // graph-key id of this hierarchy's buffers
    int coarse_hint = 0;
    long coarse_iters = 0;     // coarse BiCGStab iterations of the last solve
    ~lq_mg()
    {
        if (chsc) (void)hipHostFree(chsc);
        if (ohsc) (void)hipHostFree(ohsc);
    }
};

namespace lq {
namespace {

long g_mg_ids = 0;

FieldView full32(const lq_mg *mg, char *base)
{
    return FieldView{base, F32, (long)mg->m.g.vh, fb(F32, mg->m.g), 2};
}
FieldView full64(const lq_mg *mg, char *base)
{
    return FieldView{base, F64, (long)mg->m.g.vh, fb(F64, mg->m.g), 2};
}
char *fine32(lq_mg *mg, int i) { return mg->fws.ptr + (size_t)i * 2 * fb(F32, mg->m.g); }
char *fine64(lq_mg *mg, int i) { return mg->f64ws.ptr + (size_t)i * 2 * fb(F64, mg->m.g); }
char *cvec(lq_mg *mg, int i) { return mg->cws.ptr + (size_t)i * mg->cbytes; }
dim3 fine_grid(const lq_mg *mg) { return dim3((unsigned)((mg->m.g.vh + MT - 1) / MT), 2); }
int fine_nb(const lq_mg *mg) { return (mg->m.g.vh + MT - 1) / MT; }

void coarse_apply_fn(SolveCtx &c, const FieldView &out, const FieldView &in)
{
    const lq_mg *mg = static_cast<const lq_mg *>(c.coarse);
    mg_capply_kernel<<<mg->m.nagg, MT, 0, c.s>>>(mg->m, reinterpret_cast<const float2 *>(mg->dc.ptr), in.base,
                                                 out.base, c.masked ? c.sc : nullptr);
    LQ_HIP(hipGetLastError());
}

SolveCtx coarse_ctx(lq_mg *mg, hipStream_t s)
{
    SolveCtx c;
    c.op = mg->op;
    c.s = s;
    c.nsys = 1;
    c.eo = false;
    c.sps = 1;
    c.pin = F32;
    c.px = F32;
    c.sc = reinterpret_cast<double *>(mg->csc.ptr);
    c.hsc = mg->chsc;
    c.partial = reinterpret_cast<double *>(mg->cpart.ptr);
    const auto v = [&](int i) { return FieldView{cvec(mg, i), F32, mg->npseudo, mg->cbytes, 1}; };
    c.irin = v(0);
    c.ix = v(1);
    c.ir = v(2);
    c.ip = v(3);
    c.iv = v(4);
    c.is = v(5);
    c.it = v(6);
    c.irhat = v(7);
    c.iw = v(8);
    c.ex = v(9);
    c.coarse_apply = coarse_apply_fn;
    c.coarse = mg;
    c.key_extra = mg->id;
    return c;
}

// |x|^2 of an FP32 or FP64 full field, summed on the host in a fixed order
double norm2_full(lq_mg *mg, const FieldView &x, hipStream_t s)
{
    const int nb = blas_blocks(x.n);
    LQ_HIP(launch_reduce(x, x, RED_NORM, reinterpret_cast<double *>(mg->part.ptr), s));
    mg->hpart.resize(2 * (size_t)nb);
    LQ_HIP(hipMemcpyAsync(mg->hpart.data(), mg->part.ptr, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
    double t = 0;
    for (int i = 0; i < 2 * nb; ++i) t += mg->hpart[i];
    return t;
}

// <X_j, x> for j < nx (X: FP32 full fields xstride bytes apart), host sums
void mdot_full(lq_mg *mg, const char *X, long xstride, int nx, const FieldView &x, std::vector<double> &out,
               hipStream_t s)
{
    const int nb = fine_nb(mg);
    mg_mdot_kernel<<<dim3(nb, 2, (nx + 7) / 8), MT, 0, s>>>(X, xstride, nx, x,
                                                           reinterpret_cast<double *>(mg->part.ptr));
    LQ_HIP(hipGetLastError());
    const size_t np = (size_t)nx * 2 * nb * 2;
    mg->hpart.resize(np);
    LQ_HIP(hipMemcpyAsync(mg->hpart.data(), mg->part.ptr, sizeof(double) * np, hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
    out.assign(2 * (size_t)nx, 0.0);
    for (int j = 0; j < nx; ++j)
        for (int sl = 0; sl < 2; ++sl)
            for (int b = 0; b < nb; ++b) {
                const double *p = mg->hpart.data() + (((size_t)j * 2 + sl) * nb + b) * 2;
                out[2 * j] += p[0];
                out[2 * j + 1] += p[1];
            }
}

// z = K r: coarse correction P D_c^-1 P^dag r, then smooth_steps
// minimal-residual steps on r - D z (FP32 full fields)
void mg_cycle(lq_mg *mg, const FieldView &r, const FieldView &z, hipStream_t s)
{
    const MgGeom &m = mg->m;
    SolveCtx c = coarse_ctx(mg, s);
    mg_restrict_kernel<<<m.nagg, MT, 0, s>>>(m, mg->vecs.ptr, r.base, c.irin.base);
    LQ_HIP(hipGetLastError());
    std::memset(c.hsc, 0, sizeof(double) * NSC);
    c.hsc[SC_TARGET2] = mg->prm.coarse_tol * mg->prm.coarse_tol;
    c.push();
    mg->coarse_iters += bicgstab_solve(c, mg->prm.coarse_max_iter, 8, mg->coarse_hint);
    mg_prolong_kernel<<<fine_grid(mg), MT, 0, s>>>(m, mg->vecs.ptr, c.ix.base, z.base);
    LQ_HIP(hipGetLastError());
    if (mg->prm.smooth_steps <= 0) return;
    lq_op *op = mg->op;
    const int M = mg->prm.gcr_restart;
    const FieldView sv = full32(mg, fine32(mg, 2 * M + 2)), q = full32(mg, fine32(mg, 2 * M + 3)),
                    d = full32(mg, fine32(mg, 2 * M + 4)), t = full32(mg, fine32(mg, 2 * M + 5));
    dirac_full(op, F32, t.base, z.base, 1, false, s);
    mg_smooth_init_kernel<<<fine_grid(mg), MT, 0, s>>>(sv, r, t, d);
    LQ_HIP(hipGetLastError());
    double *ssc = reinterpret_cast<double *>(mg->osc.ptr) + NSC;
    const int nb = fine_nb(mg);
    for (int it = 0; it < mg->prm.smooth_steps; ++it) {
        dirac_full(op, F32, q.base, sv.base, 1, false, s);
        LQ_HIP(launch_reduce(sv, q, RED_DOT_NORM, reinterpret_cast<double *>(mg->part.ptr), s));
        LQ_HIP(launch_finish(reinterpret_cast<double *>(mg->part.ptr), 1, 2, nb, 3, FIN_BICG_OMEGA, ssc, 1e-30, s));
        mg_mr_kernel<<<fine_grid(mg), MT, 0, s>>>(d, sv, q, ssc);
        LQ_HIP(hipGetLastError());
    }
    mg_add_kernel<<<fine_grid(mg), MT, 0, s>>>(z, d);
    LQ_HIP(hipGetLastError());
}

// Flexible GCR on D e = r (FP32 full fields; r is overwritten with the
// residual) to |r|^2 <= rel^2 |r_0|^2 or max_it iterations; returns the
// iterations.
int mg_gcr(lq_mg *mg, const FieldView &r, const FieldView &e, double rel, int max_it, hipStream_t s)
{
    const int M = mg->prm.gcr_restart;
    const long vs = 2 * fb(F32, mg->m.g);
    char *Z = fine32(mg, 0), *W = fine32(mg, M);
    LQ_HIP(launch_zero(e, s));
    const double rr0 = norm2_full(mg, r, s);
    if (!(rr0 > 0)) return 0;
    double rr = rr0;
    std::vector<double> ww(M), dots;
    int it = 0;
    const int nb = fine_nb(mg);
    while (it < max_it && rr > rel * rel * rr0) {
        for (int i = 0; i < M && it < max_it && rr > rel * rel * rr0; ++i, ++it) {
            const FieldView zi = full32(mg, Z + i * vs), wi = full32(mg, W + i * vs);
            mg_cycle(mg, r, zi, s);
            dirac_full(mg->op, F32, wi.base, zi.base, 1, false, s);
            // classical Gram-Schmidt against the previous w_j, twice
            for (int pass = 0; pass < 2 && i > 0; ++pass) {
                mdot_full(mg, W, vs, i, wi, dots, s);
                std::vector<double> cf(2 * (size_t)i);
                for (int j = 0; j < i; ++j) {
                    cf[2 * j] = dots[2 * j] / ww[j];
                    cf[2 * j + 1] = dots[2 * j + 1] / ww[j];
                }
                LQ_HIP(hipMemcpyAsync(mg->coef.ptr, cf.data(), sizeof(double) * cf.size(), hipMemcpyHostToDevice, s));
                mg_maxpy_kernel<<<fine_grid(mg), MT, 0, s>>>(wi, W, vs, i, reinterpret_cast<double *>(mg->coef.ptr));
                LQ_HIP(hipGetLastError());
                mg_maxpy_kernel<<<fine_grid(mg), MT, 0, s>>>(zi, Z, vs, i, reinterpret_cast<double *>(mg->coef.ptr));
                LQ_HIP(hipGetLastError());
            }
            ww[i] = norm2_full(mg, wi, s);
            if (!(ww[i] > 0) || !std::isfinite(ww[i])) throw Failure{LQ_ERR_NONFINITE, "multigrid GCR: breakdown"};
            mdot_full(mg, W + i * vs, vs, 1, r, dots, s);  // <w_i, r>
            const double ar = dots[0] / ww[i], ai = dots[1] / ww[i];
            mg_gcr_update_kernel<<<fine_grid(mg), MT, 0, s>>>(e, zi, r, wi, ar, ai,
                                                              reinterpret_cast<double *>(mg->part.ptr));
            LQ_HIP(hipGetLastError());
            mg->hpart.resize(2 * (size_t)nb);
            LQ_HIP(hipMemcpyAsync(mg->hpart.data(), mg->part.ptr, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, s));
            LQ_HIP(hipStreamSynchronize(s));
            rr = 0;
            for (int b = 0; b < 2 * nb; ++b) rr += mg->hpart[b];
            if (!std::isfinite(rr)) throw Failure{LQ_ERR_NONFINITE, "multigrid GCR: residual is not finite"};
        }
    }
    return it;
}

void build_coarse(lq_mg *mg, hipStream_t s)
{
    const MgGeom &m = mg->m;
    constexpr int CH = 16;  // columns per multi-RHS apply
    const int ncol_max = std::min(CH, m.n2);
    const long zs = 2 * fb(F64, m.g);
    Buf zbuf, wbuf;
    zbuf.ensure((size_t)ncol_max * zs);
    wbuf.ensure((size_t)ncol_max * zs);
    for (int color = 0; color < 16; ++color)
        for (int col0 = 0; col0 < m.n2; col0 += CH) {
            const int ncol = std::min(CH, m.n2 - col0);
            mg_column_kernel<<<dim3((unsigned)((m.g.vh + MT - 1) / MT), 2), MT, 0, s>>>(m, mg->vecs.ptr, color, col0,
                                                                                        ncol, zbuf.ptr, zs);
            LQ_HIP(hipGetLastError());
            dirac_full(mg->op, F64, wbuf.ptr, zbuf.ptr, ncol, false, s);
            const size_t lds = sizeof(float2) * (size_t)(m.nv + ncol) * BC * 12 + sizeof(int) * BC;
            mg_build_kernel<<<m.nagg, MT, lds, s>>>(m, mg->vecs.ptr, wbuf.ptr, zs, color, col0, ncol,
                                                    reinterpret_cast<float2 *>(mg->dc.ptr));
            LQ_HIP(hipGetLastError());
        }
    LQ_HIP(hipStreamSynchronize(s));  // zbuf, wbuf are freed on return
}

std::string check_mg_params(const lq_op *op, const lq_mg_params *p)
{
    for (int mu = 0; mu < 4; ++mu) {
        const int b = p->block[mu], L = op->g.L[mu];
        if (b < 2 || L % b || (L / b) % 2 || L / b < 2)
            return "every block extent must be >= 2 and divide L with an even quotient >= 2";
    }
    if (p->nvec < 1 || p->nvec > 32) return "nvec must be in [1, 32]";
    if (p->setup_iters < 0 || !(p->setup_tol > 0) || !(p->setup_tol < 1)) return "setup_iters or setup_tol out of range";
    if (p->smooth_steps < 0 || !(p->coarse_tol > 0) || !(p->coarse_tol < 1) || p->coarse_max_iter < 1)
        return "smooth_steps, coarse_tol or coarse_max_iter out of range";
    if (p->gcr_restart < 1 || p->gcr_restart > 32) return "gcr_restart must be in [1, 32]";
    return "";
}

}  // namespace
}  // namespace lq

extern "C" {

void lq_mg_params_default(lq_mg_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    for (int mu = 0; mu < 4; ++mu) p->block[mu] = 4;
    p->nvec = 12;
    p->setup_iters = 3;
    p->setup_tol = 1e-2;
    p->smooth_steps = 8;
    p->coarse_tol = 0.2;
    p->coarse_max_iter = 200;
    p->gcr_restart = 16;
}

lq_status lq_mg_create(lq_op *op, const lq_mg_params *p, const void *v0, lq_mg **out, void *stream)
{
    if (!op || !p || !v0 || !out) {
        set_error("lq_mg_create: null argument");
        return LQ_ERR_ARG;
    }
    *out = nullptr;
    const std::string why = check_mg_params(op, p);
    if (!why.empty()) {
        set_error("lq_mg_create: " + why);
        return LQ_ERR_ARG;
    }
    if (!op->gauge_set) {
        set_error("lq_mg_create: gauge field not set");
        return LQ_ERR_STATE;
    }
    lq_mg *mg = new lq_mg;
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t us = static_cast<hipStream_t>(stream);
        LQ_HIP(hipEventRecord(op->ev_in, us));
        LQ_HIP(hipStreamWaitEvent(op->stream, op->ev_in, 0));
        hipStream_t s = op->stream;
        mg->op = op;
        mg->prm = *p;
        mg->id = ++g_mg_ids;
        MgGeom &m = mg->m;
        m.g = op->g;
        m.nagg = 1;
        m.asz = 1;
        for (int mu = 0; mu < 4; ++mu) {
            m.bl[mu] = p->block[mu];
            m.lc[mu] = op->g.L[mu] / p->block[mu];
            m.nagg *= m.lc[mu];
            m.asz *= m.bl[mu];
        }
        m.nv = p->nvec;
        m.n2 = 2 * p->nvec;
        m.vstride = 2 * fb(F32, m.g);
        mg->npseudo = ((long)m.nagg * m.n2 + 11) / 12;
        mg->cbytes = (spinor_field_bytes(F32, mg->npseudo) + 255) & ~255L;
        const int M = p->gcr_restart;
        mg->vecs.ensure((size_t)m.nv * m.vstride);
        mg->dc.ensure(sizeof(float2) * (size_t)m.nagg * 9 * m.n2 * m.n2);
        mg->cws.ensure(10 * (size_t)mg->cbytes);
        LQ_HIP(hipMemsetAsync(mg->cws.ptr, 0, 10 * (size_t)mg->cbytes, s));  // pseudo-site tails stay zero
        mg->csc.ensure(sizeof(double) * NSC);
        mg->cpart.ensure(sizeof(double) * 3 * (size_t)blas_blocks(mg->npseudo) * 2);
        LQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&mg->chsc), sizeof(double) * NSC, 0));
        LQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&mg->ohsc), sizeof(double) * 2 * NSC, 0));
        mg->fws.ensure((size_t)(2 * M + 6) * 2 * fb(F32, m.g));
        mg->f64ws.ensure(4 * 2 * (size_t)fb(F64, m.g));
        const int nb = fine_nb(mg);
        mg->part.ensure(sizeof(double) * std::max<size_t>(3 * 2 * (size_t)nb, (size_t)32 * 2 * nb * 2));
        mg->coef.ensure(sizeof(double) * 2 * 32);
        mg->osc.ensure(sizeof(double) * 2 * NSC);
        LQ_HIP(hipMemsetAsync(mg->osc.ptr, 0, sizeof(double) * 2 * NSC, s));
        // near-null vectors: v0, improved by inverse iterations with the
        // operator's own solver, normalised, in FP32; the vectors are solved
        // together as one multi-RHS solve (in groups that fit an operator
        // bound to a workspace of fewer right-hand sides)
        lq_solver_params sp;
        lq_solver_params_default(&sp);
        sp.tol = p->setup_tol;
        sp.inner = LQ_F32;
        sp.inner_tol = std::max(1e-5, p->setup_tol * 0.1);
        const long vlex = (long)m.g.vh * 2 * 12 * 2;  // doubles of one complex128 full field
        const int grp = op->bound_nrhs ? std::min(m.nv, op->bound_nrhs) : m.nv;
        const size_t ffb = 2 * (size_t)fb(F64, m.g);  // bytes of one packed FP64 full field
        Buf sws, ssc, spart;                          // freed when the set-up ends
        if (p->setup_iters > 0) {
            sws.ensure(2 * ffb * grp);
            ssc.ensure(sizeof(double) * NSC * grp);
            spart.ensure(sizeof(double) * 2 * (size_t)grp * blas_blocks(m.g.vh));
            LQ_HIP(hipMemsetAsync(ssc.ptr, 0, sizeof(double) * NSC * grp, s));
        }
        double *osc = reinterpret_cast<double *>(ssc.ptr);
        for (int k0 = 0; k0 < m.nv; k0 += grp) {
            const int n = std::min(grp, m.nv - k0);
            char *bp = p->setup_iters > 0 ? sws.ptr : fine64(mg, 0);
            char *xp = p->setup_iters > 0 ? sws.ptr + ffb * grp : fine64(mg, 1);
            const int nb_ = p->setup_iters > 0 ? n : 1;
            for (int k = k0; k < k0 + n; ++k) {
                char *dst = p->setup_iters > 0 ? bp + ffb * (k - k0) : bp;
                for (int par = 0; par < 2; ++par)
                    LQ_HIP(launch_pack_spinor(m.g, par, 0, static_cast<const double *>(v0) + k * vlex,
                                              full_parity_view(dst, F64, m.g, 1, par), s));
                if (p->setup_iters == 0)
                    LQ_HIP(launch_copy(full32(mg, mg->vecs.ptr + k * m.vstride), full64(mg, dst), nullptr, 2, false,
                                       s));
            }
            if (p->setup_iters == 0) continue;
            const FieldView bs{bp, F64, (long)m.g.vh, fb(F64, m.g), 2 * nb_};
            const FieldView xs{xp, F64, (long)m.g.vh, fb(F64, m.g), 2 * nb_};
            for (int it = 0; it < p->setup_iters; ++it) {
                std::vector<lq_solve_stats> st(n);
                const lq_status rc = solve_packed(op, sp, n, xp, bp, false, st.data(), s);
                if (rc < 0) throw Failure{rc, std::string("lq_mg_create: setup solve: ") + get_error()};
                // b = x / |x|, per vector
                LQ_HIP(launch_reduce(xs, xs, RED_NORM, reinterpret_cast<double *>(spart.ptr), s));
                LQ_HIP(launch_finish(reinterpret_cast<double *>(spart.ptr), n, 2, blas_blocks(m.g.vh), 1, FIN_NORM,
                                     osc, 0, s));
                LQ_HIP(launch_copy(bs, xs, osc, 2, true, s));
            }
            for (int k = k0; k < k0 + n; ++k)
                LQ_HIP(launch_copy(full32(mg, mg->vecs.ptr + k * m.vstride), full64(mg, bp + ffb * (k - k0)), osc, 2,
                                   false, s));
        }
        mg_orth_kernel<<<m.nagg, MT, 0, s>>>(m, mg->vecs.ptr);
        LQ_HIP(hipGetLastError());
        build_coarse(mg, s);
        LQ_HIP(hipEventRecord(op->ev_out, s));
        LQ_HIP(hipStreamWaitEvent(us, op->ev_out, 0));
        LQ_HIP(hipStreamSynchronize(us));
        *out = mg;
        return LQ_OK;
    } catch (const Failure &f) {
        delete mg;
        set_error(f.msg);
        return f.code;
    } catch (const std::exception &e) {
        delete mg;
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}

lq_status lq_mg_destroy(lq_mg *mg)
{
    if (!mg) return LQ_OK;
    try {
        LQ_HIP(hipSetDevice(mg->op->device));
        LQ_HIP(hipDeviceSynchronize());
        mg->op->clear_graphs();  // the coarse solver's captured chunks read this hierarchy's buffers
    } catch (const Failure &f) {
        set_error(f.msg);
        delete mg;
        return f.code;
    }
    delete mg;
    return LQ_OK;
}

lq_status lq_mg_solve(lq_mg *mg, const lq_solver_params *sp, void *x, const void *b, lq_solve_stats *stats,
                      void *stream)
{
    if (!mg || !sp || !x || !b) {
        set_error("lq_mg_solve: null argument");
        return LQ_ERR_ARG;
    }
    if (!(sp->tol > 0) || !(sp->inner_tol > 0) || !(sp->inner_tol < 1) || sp->max_iter < 0 || sp->max_outer < 0) {
        set_error("lq_mg_solve: tol, inner_tol, max_iter or max_outer out of range");
        return LQ_ERR_ARG;
    }
    lq_op *op = mg->op;
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t us = static_cast<hipStream_t>(stream);
        LQ_HIP(hipEventRecord(op->ev_in, us));
        LQ_HIP(hipStreamWaitEvent(op->stream, op->ev_in, 0));
        hipStream_t s = op->stream;
        const auto t0 = std::chrono::steady_clock::now();
        const MgGeom &m = mg->m;
        const int M = mg->prm.gcr_restart;
        const FieldView b64 = full64(mg, fine64(mg, 0)), x64 = full64(mg, fine64(mg, 1)),
                        r64 = full64(mg, fine64(mg, 2)), t64 = full64(mg, fine64(mg, 3));
        const FieldView r32 = full32(mg, fine32(mg, 2 * M)), e32 = full32(mg, fine32(mg, 2 * M + 1));
        for (int par = 0; par < 2; ++par)
            LQ_HIP(launch_pack_spinor(m.g, par, 0, static_cast<const double *>(b),
                                      full_parity_view(b64.base, F64, m.g, 1, par), s));
        LQ_HIP(launch_zero(x64, s));
        double *osc = reinterpret_cast<double *>(mg->osc.ptr);
        const double bn2 = norm2_full(mg, b64, s);
        if (!std::isfinite(bn2)) throw Failure{LQ_ERR_NONFINITE, "right-hand side is not finite"};
        const double target = sp->tol * sp->tol * bn2;
        int iters = 0, outer = 0;
        double r2 = bn2;
        mg->coarse_iters = 0;
        const int nb = blas_blocks(m.g.vh);
        for (int step = 0; step <= sp->max_outer; ++step) {
            // r = b - D x in FP64 (b itself for the zero start) and |r|^2
            if (step == 0) {
                LQ_HIP(launch_copy(r64, b64, osc, 2, false, s));
                LQ_HIP(launch_reduce(r64, r64, RED_NORM, reinterpret_cast<double *>(mg->part.ptr), s));
            } else {
                dirac_full(op, F64, t64.base, x64.base, 1, false, s);
                LQ_HIP(launch_xmy_norm(r64, b64, t64, reinterpret_cast<double *>(mg->part.ptr), s));
            }
            LQ_HIP(launch_finish(reinterpret_cast<double *>(mg->part.ptr), 1, 2, nb, 1, FIN_NORM, osc, 0, s));
            LQ_HIP(hipMemcpyAsync(mg->ohsc, osc, sizeof(double) * NSC, hipMemcpyDeviceToHost, s));
            LQ_HIP(hipStreamSynchronize(s));
            r2 = mg->ohsc[SC_NORM2];
            if (!std::isfinite(r2)) throw Failure{LQ_ERR_NONFINITE, "residual is not finite"};
            if (r2 <= target || step == sp->max_outer || iters >= sp->max_iter) break;
            ++outer;
            double rel = 0.5 * std::sqrt(target / r2);
            rel = std::min(0.5, std::max(rel, sp->inner_tol));
            LQ_HIP(launch_copy(r32, r64, osc, 2, true, s));  // r / |r|
            iters += mg_gcr(mg, r32, e32, rel, sp->max_iter - iters, s);
            LQ_HIP(launch_accum(x64, e32, osc, 2, true, s));  // x += |r| e
        }
        for (int par = 0; par < 2; ++par)
            LQ_HIP(launch_unpack_spinor(m.g, par, 0, full_parity_view(x64.base, F64, m.g, 1, par),
                                        static_cast<double *>(x), s));
        LQ_HIP(hipEventRecord(op->ev_out, s));
        LQ_HIP(hipStreamWaitEvent(us, op->ev_out, 0));
        LQ_HIP(hipStreamSynchronize(us));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        const double diff = bn2 > 0 ? std::sqrt(r2 / bn2) : 0.0;
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            stats->nconv = iters;
            stats->nouter = outer;
            stats->converged = diff <= sp->tol ? 1 : 0;
            stats->diff = diff;
            stats->t_solve_ms = ms;
        }
        if (log_level(op) >= 1)
            std::fprintf(stderr, "lq: multigrid solve: %d outer steps, %d GCR iterations, %ld coarse iterations, "
                                 "|r| / |b| %.3e\n", outer, iters, mg->coarse_iters, diff);
        return diff <= sp->tol ? LQ_OK : LQ_NOT_CONVERGED;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}

lq_status lq_mg_vectors(const lq_mg *mg, void *out, void *stream)
{
    if (!mg || !out) {
        set_error("lq_mg_vectors: null argument");
        return LQ_ERR_ARG;
    }
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        const MgGeom &m = mg->m;
        const long vlex = (long)m.g.vh * 2 * 12 * 2;
        for (int k = 0; k < m.nv; ++k)
            for (int par = 0; par < 2; ++par)
                LQ_HIP(launch_unpack_spinor(m.g, par, 0,
                                            full_parity_view(mg->vecs.ptr + k * m.vstride, F32, m.g, 1, par),
                                            static_cast<double *>(out) + k * vlex, s));
        LQ_HIP(hipStreamSynchronize(s));
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}

lq_status lq_mg_coarse_op(const lq_mg *mg, double *out)
{
    if (!mg || !out) {
        set_error("lq_mg_coarse_op: null argument");
        return LQ_ERR_ARG;
    }
    try {
        const size_t n = (size_t)mg->m.nagg * 9 * mg->m.n2 * mg->m.n2;
        std::vector<float> h(2 * n);
        LQ_HIP(hipMemcpy(h.data(), mg->dc.ptr, sizeof(float) * 2 * n, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < 2 * n; ++i) out[i] = h[i];
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}

lq_status lq_mg_restrict(lq_mg *mg, const void *fine, void *coarse, void *stream)
{
    if (!mg || !fine || !coarse) {
        set_error("lq_mg_restrict: null argument");
        return LQ_ERR_ARG;
    }
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        const MgGeom &m = mg->m;
        const FieldView f = full32(mg, fine32(mg, 2 * mg->prm.gcr_restart));
        char *tmp64 = fine64(mg, 3);
        for (int par = 0; par < 2; ++par)
            LQ_HIP(launch_pack_spinor(m.g, par, 0, static_cast<const double *>(fine),
                                      full_parity_view(tmp64, F64, m.g, 1, par), s));
        LQ_HIP(launch_copy(f, full64(mg, tmp64), nullptr, 2, false, s));
        mg_restrict_kernel<<<m.nagg, MT, 0, s>>>(m, mg->vecs.ptr, f.base, cvec(mg, 0));
        LQ_HIP(hipGetLastError());
        const long n = (long)m.nagg * m.n2;
        mg_cexport_kernel<<<(unsigned)((n + MT - 1) / MT), MT, 0, s>>>(n, cvec(mg, 0), static_cast<double *>(coarse));
        LQ_HIP(hipGetLastError());
        LQ_HIP(hipStreamSynchronize(s));
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}

lq_status lq_mg_prolong(lq_mg *mg, const void *coarse, void *fine, void *stream)
{
    if (!mg || !fine || !coarse) {
        set_error("lq_mg_prolong: null argument");
        return LQ_ERR_ARG;
    }
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        const MgGeom &m = mg->m;
        const long n = (long)m.nagg * m.n2;
        mg_cimport_kernel<<<(unsigned)((n + MT - 1) / MT), MT, 0, s>>>(n, static_cast<const double *>(coarse),
                                                                       cvec(mg, 0));
        LQ_HIP(hipGetLastError());
        const FieldView f = full32(mg, fine32(mg, 2 * mg->prm.gcr_restart));
        mg_prolong_kernel<<<fine_grid(mg), MT, 0, s>>>(m, mg->vecs.ptr, cvec(mg, 0), f.base);
        LQ_HIP(hipGetLastError());
        char *tmp64 = fine64(mg, 3);
        LQ_HIP(launch_copy(full64(mg, tmp64), f, nullptr, 2, false, s));
        for (int par = 0; par < 2; ++par)
            LQ_HIP(launch_unpack_spinor(m.g, par, 0, full_parity_view(tmp64, F64, m.g, 1, par),
                                        static_cast<double *>(fine), s));
        LQ_HIP(hipStreamSynchronize(s));
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}

lq_status lq_mg_coarse_apply(lq_mg *mg, const void *xin, void *yout, void *stream)
{
    if (!mg || !xin || !yout) {
        set_error("lq_mg_coarse_apply: null argument");
        return LQ_ERR_ARG;
    }
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        const MgGeom &m = mg->m;
        const long n = (long)m.nagg * m.n2;
        mg_cimport_kernel<<<(unsigned)((n + MT - 1) / MT), MT, 0, s>>>(n, static_cast<const double *>(xin),
                                                                       cvec(mg, 0));
        LQ_HIP(hipGetLastError());
        mg_capply_kernel<<<m.nagg, MT, 0, s>>>(m, reinterpret_cast<const float2 *>(mg->dc.ptr), cvec(mg, 0),
                                               cvec(mg, 1), nullptr);
        LQ_HIP(hipGetLastError());
        mg_cexport_kernel<<<(unsigned)((n + MT - 1) / MT), MT, 0, s>>>(n, cvec(mg, 1), static_cast<double *>(yout));
        LQ_HIP(hipGetLastError());
        LQ_HIP(hipStreamSynchronize(s));
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}

}  // extern "C"
