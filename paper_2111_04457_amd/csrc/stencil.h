// stencil.h -- per-site pieces of the hopping term of eq. (1) (Sec. 3) and
// of the clover term, shared by the operator, force and batch kernels.
#pragma once

#include "lq_common.h"

namespace lq {

// h = psi_up + s B psi_dn, B the upper-right 2x2 block of gamma_mu in the
// chiral basis: B = -i sigma_1, -i sigma_2, -i sigma_3, 1 for mu = x, y, z, t.
template <int MU, int SG, typename R>
__device__ __forceinline__ void project(const Spinor<R> &p, cx<R> h[6])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> b0, b1;  // (B psi_dn)_0, (B psi_dn)_1
        const cx<R> d2 = p.c[6 + a], d3 = p.c[9 + a];
        if constexpr (MU == 0) { b0 = tmi(d3); b1 = tmi(d2); }
        else if constexpr (MU == 1) { b0 = mk(-d3.re, -d3.im); b1 = d2; }
        else if constexpr (MU == 2) { b0 = tmi(d2); b1 = ti(d3); }
        else { b0 = d2; b1 = d3; }
        if constexpr (SG > 0) {
            h[a] = p.c[a] + b0;
            h[3 + a] = p.c[3 + a] + b1;
        } else {
            h[a] = p.c[a] - b0;
            h[3 + a] = p.c[3 + a] - b1;
        }
    }
}

// ------------------------------------------ binary16 dot-product forms --
//
// With binary16 storage the colour products run on two-way dot products of
// binary16 pairs accumulated in FP32 (each product of two binary16 values is
// exact in FP32): a complex multiply-add is two dot products instead of
// four multiply-adds.  The projection is taken in packed binary16 on the
// stored (per-site normalised, |value| <= 1) spinor, so |h| <= 2; the
// spinor's scale and the boundary phase are applied to the FP32 products.

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2 swp(h2 a) { return __builtin_shufflevector(a, a, 1, 0); }
__device__ __forceinline__ h2 neg_hi(h2 a) { return h2{a.x, -a.y}; }
__device__ __forceinline__ h2 neg_lo(h2 a) { return h2{-a.x, a.y}; }

// a.x b.x + a.y b.y + c and a.x b.x - a.y b.y + c (the sign as an operand
// modifier of the dot product), with c = 0 taken as an inline constant.
__device__ __forceinline__ float dot2(h2 a, h2 b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }
__device__ __forceinline__ float dot2_0(h2 a, h2 b)
{
    float d;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(d) : "v"(a), "v"(b));
    return d;
}
__device__ __forceinline__ float dot2n(h2 a, h2 b, float c)
{
    float d;
    asm("v_dot2_f32_f16 %0, %1, %2, %3 neg_hi:[0,1,0]" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}
__device__ __forceinline__ float dot2n_0(h2 a, h2 b)
{
    float d;
    asm("v_dot2_f32_f16 %0, %1, %2, 0 neg_hi:[0,1,0]" : "=v"(d) : "v"(a), "v"(b));
    return d;
}

// The projected half spinor h = psi_up + s B psi_dn as (re, im) pairs, and
// hs = (im, re) (one packed add each; the swaps and negations of B are
// operand modifiers).
template <int MU, int SG>
__device__ __forceinline__ void project_h2(const h2 p[12], h2 h[6], h2 hs[6])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h2 b0, b1;  // (s B psi_dn)_0, (s B psi_dn)_1 as (re, im)
        const h2 d2 = p[6 + a], d3 = p[9 + a];
        // -i d = (d.im, -d.re), i d = (-d.im, d.re)
        if constexpr (MU == 0) { b0 = neg_hi(swp(d3)); b1 = neg_hi(swp(d2)); }
        else if constexpr (MU == 1) { b0 = -d3; b1 = d2; }
        else if constexpr (MU == 2) { b0 = neg_hi(swp(d2)); b1 = neg_lo(swp(d3)); }
        else { b0 = d2; b1 = d3; }
        if constexpr (SG < 0) { b0 = -b0; b1 = -b1; }
        const h2 u0 = p[a], u1 = p[3 + a];
        h[a] = u0 + b0;
        h[3 + a] = u1 + b1;
        hs[a] = swp(u0) + swp(b0);
        hs[3 + a] = swp(u1) + swp(b1);
    }
}

// o = U h (DAGU = false) or U^dag h for the two spin rows, U as binary16
// (re, im) pairs.  U h: re = sum Ur hr - Ui hi = <u, h> with the second
// product negated, im = sum Ur hi + Ui hr = <u, hs>; U^dag h: re = <u, h>,
// im = sum Ur hi - Ui hr = <u, hs> with the second product negated.
template <bool DAGU>
__device__ __forceinline__ void su3_mul_h2(const h2 u[9], const h2 h[6], const h2 hs[6], cx<float> o[6])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re, im;
            if constexpr (!DAGU) {
                re = dot2n_0(u[a * 3], h[s * 3]);
                im = dot2_0(u[a * 3], hs[s * 3]);
#pragma unroll
                for (int b = 1; b < 3; ++b) {
                    re = dot2n(u[a * 3 + b], h[s * 3 + b], re);
                    im = dot2(u[a * 3 + b], hs[s * 3 + b], im);
                }
            } else {
                re = dot2_0(u[a], h[s * 3]);
                im = dot2n_0(u[a], hs[s * 3]);
#pragma unroll
                for (int b = 1; b < 3; ++b) {
                    re = dot2(u[b * 3 + a], h[s * 3 + b], re);
                    im = dot2n(u[b * 3 + a], hs[s * 3 + b], im);
                }
            }
            o[s * 3 + a] = mk(re, im);
        }
}

// acc += sc (u, s B^dag u): reconstruct with the spinor's scale folded in.
template <int MU, int SG>
__device__ __forceinline__ void reconstruct_sc(cx<float> acc[12], const cx<float> u[6], float sc)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<float> u0 = u[a], u1 = u[3 + a];
        cx<float> l0, l1;  // (B^dag u)_0, (B^dag u)_1
        if constexpr (MU == 0) { l0 = ti(u1); l1 = ti(u0); }
        else if constexpr (MU == 1) { l0 = u1; l1 = mk(-u0.re, -u0.im); }
        else if constexpr (MU == 2) { l0 = ti(u0); l1 = tmi(u1); }
        else { l0 = u0; l1 = u1; }
        if constexpr (SG < 0) { l0 = mk(-l0.re, -l0.im); l1 = mk(-l1.re, -l1.im); }
        acc[a] = mk(fmar(u0.re, sc, acc[a].re), fmar(u0.im, sc, acc[a].im));
        acc[3 + a] = mk(fmar(u1.re, sc, acc[3 + a].re), fmar(u1.im, sc, acc[3 + a].im));
        acc[6 + a] = mk(fmar(l0.re, sc, acc[6 + a].re), fmar(l0.im, sc, acc[6 + a].im));
        acc[9 + a] = mk(fmar(l1.re, sc, acc[9 + a].re), fmar(l1.im, sc, acc[9 + a].im));
    }
}

// acc += (u, s B^dag u) with u the colour-multiplied half spinor.
template <int MU, int SG, typename R>
__device__ __forceinline__ void reconstruct(cx<R> acc[12], const cx<R> u[6])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<R> u0 = u[a], u1 = u[3 + a];
        cx<R> l0, l1;  // (B^dag u)_0, (B^dag u)_1
        if constexpr (MU == 0) { l0 = ti(u1); l1 = ti(u0); }
        else if constexpr (MU == 1) { l0 = u1; l1 = mk(-u0.re, -u0.im); }
        else if constexpr (MU == 2) { l0 = ti(u0); l1 = tmi(u1); }
        else { l0 = u0; l1 = u1; }
        acc[a] = acc[a] + u0;
        acc[3 + a] = acc[3 + a] + u1;
        if constexpr (SG > 0) {
            acc[6 + a] = acc[6 + a] + l0;
            acc[9 + a] = acc[9 + a] + l1;
        } else {
            acc[6 + a] = acc[6 + a] - l0;
            acc[9 + a] = acc[9 + a] - l1;
        }
    }
}

// Load link (parity p, direction mu, site cb) as 9 complex numbers.
template <int P, int NL>
__device__ __forceinline__ void load_link(const char *__restrict__ links, int vh, int p, int mu, int cb,
                                          cx<typename PT<P>::R> u[9])
{
    using S = typename PT<P>::S;
    using R = typename PT<P>::R;
    const char *base = links + (long)(p * 4 + mu) * Planes<S, NL>::field_bytes(vh);
    S raw[NL];
    load_planes<S, NL>(base, cb, vh, raw);
#pragma unroll
    for (int i = 0; i < NL / 2; ++i) u[i] = cx<R>{(R)raw[2 * i], (R)raw[2 * i + 1]};
    if constexpr (NL == 12) {
        // third row of an SU(3) matrix: conj(row0 x row1)
        u[6] = conj(u[1] * u[5] - u[2] * u[4]);
        u[7] = conj(u[2] * u[3] - u[0] * u[5]);
        u[8] = conj(u[0] * u[4] - u[1] * u[3]);
    }
}

// out = U h (dag = false) or U^dag h, for the two spin rows of h.
template <bool DAGU, typename R>
__device__ __forceinline__ void su3_mul(const cx<R> u[9], const cx<R> h[6], cx<R> o[6])
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> acc;
            if constexpr (!DAGU) {
                acc = u[a * 3 + 0] * h[s * 3 + 0];
                acc = cmac(acc, u[a * 3 + 1], h[s * 3 + 1]);
                acc = cmac(acc, u[a * 3 + 2], h[s * 3 + 2]);
            } else {
                acc = cmulc(u[0 * 3 + a], h[s * 3 + 0]);
                acc = cmacc(acc, u[1 * 3 + a], h[s * 3 + 1]);
                acc = cmacc(acc, u[2 * 3 + a], h[s * 3 + 2]);
            }
            o[s * 3 + a] = acc;
        }
}

// y_i += l x_j and y_j += conj(l) x_i for one strictly-lower entry l of a
// Hermitian block.  Fused in single precision, separate products in double
// (the forms the register allocator handles best for each type; both are
// the same in every kernel that uses them).
template <typename R>
__device__ __forceinline__ void clov_acc(cx<R> &yi, cx<R> &yj, const cx<R> l, const cx<R> xi, const cx<R> xj)
{
    if constexpr (sizeof(R) == 4) {
        yi = cmac(yi, l, xj);
        yj = cmacc(yj, l, xi);
    } else {
        yi = yi + l * xj;
        yj = yj + cmulc(l, xi);
    }
}

// y = C x with C two packed 6x6 Hermitian blocks: per block 6 real diagonal
// entries then the 15 strictly-lower entries (row-major) as complex pairs,
// the 72 reals already loaded (one load of the clover block can serve
// several right-hand sides).
template <typename S, typename R>
__device__ __forceinline__ void clover_mul_raw(const S *__restrict__ raw, Spinor<R> &v)
{
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const S *c = raw + 36 * b;
        cx<R> x[6], y[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) x[i] = v.c[6 * b + i];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if constexpr (sizeof(S) == 2) y[i] = mk(mul16((R)c[i], x[i].re), mul16((R)c[i], x[i].im));
            else y[i] = (R)c[i] * x[i];
        }
        int k = 6;
#pragma unroll
        for (int i = 1; i < 6; ++i)
#pragma unroll
            for (int j = 0; j < i; ++j) {
                const cx<R> l = cx<R>{(R)c[k], (R)c[k + 1]};
                k += 2;
                clov_acc(y[i], y[j], l, x[i], x[j]);
            }
#pragma unroll
        for (int i = 0; i < 6; ++i) v.c[6 * b + i] = y[i];
    }
}

// The same product loading the block of site cb.
template <int P>
__device__ __forceinline__ void clover_mul(const char *__restrict__ clov, int vh, int cb,
                                           Spinor<typename PT<P>::R> &v)
{
    typename PT<P>::S raw[72];
    load_planes<typename PT<P>::S, 72>(clov, cb, vh, raw);
    clover_mul_raw(raw, v);
}

}  // namespace lq
