// dslash_impl.h -- hopping term of eq. (1) (Sec. 3) on one parity for gfx950.
// One thread per output site; the input spinor field, links and clover are
// read through the plane layout of lq_common.h (16-byte elements, a
// wavefront reads 1 KiB contiguous per load).  Neighbour spinors are re-used
// through the L2 and the Infinity Cache; links are read exactly once.
#pragma once

#include "dslash.h"
#include "stencil.h"

namespace lq {

template <int P, int NL, bool DAG, int MU>
__device__ __forceinline__ void hop_dir(const HopArgs &a, const char *__restrict__ in, int cb, const int c[4],
                                        int p_out, cx<typename PT<P>::R> acc[12])
{
    using R = typename PT<P>::R;
    constexpr int SF = DAG ? +1 : -1;  // forward: (1 - gamma) for H, (1 + gamma) for H^dag
    constexpr int SB = -SF;
    const int vh = a.g.vh;
    {
        int d[4] = {c[0], c[1], c[2], c[3]};
        const bool wrap = (d[MU] == a.g.L[MU] - 1);
        d[MU] = wrap ? 0 : d[MU] + 1;
        const int nb = cb_index(a.g, d);
        const Spinor<R> ps = load_spinor<P>(in, nb, a.in_n);
        cx<R> h[6], u[9], o[6];
        project<MU, SF>(ps, h);
        load_link<P, NL>(a.links, vh, p_out, MU, cb, u);
        if (wrap) {
            const cx<R> ph = cx<R>{(R)a.g.bc_re[MU], (R)a.g.bc_im[MU]};
#pragma unroll
            for (int i = 0; i < 6; ++i) h[i] = ph * h[i];
        }
        su3_mul<false>(u, h, o);
        reconstruct<MU, SF>(acc, o);
    }
    {
        int d[4] = {c[0], c[1], c[2], c[3]};
        const bool wrap = (d[MU] == 0);
        d[MU] = wrap ? a.g.L[MU] - 1 : d[MU] - 1;
        const int nb = cb_index(a.g, d);
        const Spinor<R> ps = load_spinor<P>(in, nb, a.in_n);
        cx<R> h[6], u[9], o[6];
        project<MU, SB>(ps, h);
        load_link<P, NL>(a.links, vh, 1 - p_out, MU, nb, u);
        if (wrap) {
            const cx<R> ph = cx<R>{(R)a.g.bc_re[MU], -(R)a.g.bc_im[MU]};
#pragma unroll
            for (int i = 0; i < 6; ++i) h[i] = ph * h[i];
        }
        su3_mul<true>(u, h, o);
        reconstruct<MU, SB>(acc, o);
    }
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int NT>
__global__ __launch_bounds__(NT) void hop_kernel(HopArgs a)
{
    using R = typename PT<P>::R;
    // Workgroups are dispatched to the 8 XCDs round-robin; give each XCD a
    // contiguous range of (site block, rhs) tiles so that neighbour spinors
    // and, with several right-hand sides, the shared links of a site block
    // are re-read from that XCD's L2.  rhs varies fastest within the range.
    const int nbs = (a.g.vh + NT - 1) / NT;
    const int total = nbs * a.nrhs;
    const int full = a.xcd_remap ? (total / 8) * 8 : 0;
    const int id = blockIdx.x;
    const int t = id < full ? (id % 8) * (full / 8) + id / 8 : id;
    const int sblk = t / a.nrhs;
    const int rhs = t - sblk * a.nrhs;
    const int cb = sblk * NT + threadIdx.x;
    const bool valid = cb < a.g.vh;
    double red0 = 0.0, red1 = 0.0;
    if (valid) {
        const char *in = a.in + rhs * a.in_rs;
        int c[4];
        cb_coords(a.g, a.p_out, cb, c);
        cx<R> acc[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) acc[i] = cx<R>{0, 0};
        hop_dir<P, NL, DAG, 0>(a, in, cb, c, a.p_out, acc);
        hop_dir<P, NL, DAG, 1>(a, in, cb, c, a.p_out, acc);
        hop_dir<P, NL, DAG, 2>(a, in, cb, c, a.p_out, acc);
        hop_dir<P, NL, DAG, 3>(a, in, cb, c, a.p_out, acc);
        const R coef = (R)a.coef;
        Spinor<R> res;
#pragma unroll
        for (int i = 0; i < 12; ++i) res.c[i] = coef * acc[i];
        if constexpr (XPAY) {
            Spinor<R> yv = load_spinor<P>(a.y + rhs * a.y_rs, cb, a.y_n);
            if constexpr (CLOV == 1) clover_mul<P>(a.clov, a.g.vh, cb, yv);
#pragma unroll
            for (int i = 0; i < 12; ++i) res.c[i] = yv.c[i] + res.c[i];
        }
        if constexpr (CLOV == 2) clover_mul<P>(a.clov, a.g.vh, cb, res);
        store_spinor<P>(a.out + rhs * a.out_rs, cb, a.out_n, res);
        if constexpr (RED == 1) {
            // the norm of what was stored (FP16: of the rounded values)
            if constexpr (PT<P>::scaled) res = load_spinor<P>(a.out + rhs * a.out_rs, cb, a.out_n);
#pragma unroll
            for (int i = 0; i < 12; ++i) red0 += (double)norm2(res.c[i]);
        } else if constexpr (RED == 2) {
            if constexpr (PT<P>::scaled) res = load_spinor<P>(a.out + rhs * a.out_rs, cb, a.out_n);
            const Spinor<R> wv = load_spinor<P>(a.w + rhs * a.w_rs, cb, a.w_n);
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                const cx<R> t = cmulc(wv.c[i], res.c[i]);
                red0 += (double)t.re;
                red1 += (double)t.im;
            }
        }
    }
    if constexpr (RED != 0) {
        __shared__ double lds[NT / 64];
        const double s0 = block_sum<NT>(red0, lds);
        if constexpr (RED == 1) {
            if (threadIdx.x == 0) a.partial[(long)rhs * nbs + sblk] = s0;
        } else {
            const double s1 = block_sum<NT>(red1, lds);
            if (threadIdx.x == 0) {
                a.partial[2 * ((long)rhs * nbs + sblk)] = s0;
                a.partial[2 * ((long)rhs * nbs + sblk) + 1] = s1;
            }
        }
    }
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED>
static hipError_t launch_nt(const HopArgs &a, int block, hipStream_t s)
{
    const dim3 grid(hop_blocks(a.g.vh, block) * a.nrhs);
    switch (block) {
    case 64: hop_kernel<P, NL, DAG, CLOV, XPAY, RED, 64><<<grid, 64, 0, s>>>(a); break;
    case 128: hop_kernel<P, NL, DAG, CLOV, XPAY, RED, 128><<<grid, 128, 0, s>>>(a); break;
    case 256: hop_kernel<P, NL, DAG, CLOV, XPAY, RED, 256><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The epilogue combinations the operators use:
//   (clov, xpay, red) in {(0,0,0) plain hop, (2,0,0) C H x, (1,1,*) C y + c H x,
//                         (0,1,*) y + c H x, (2,1,0) C (y + c H x)}
template <int P, int NL, bool DAG>
static hipError_t launch_epi(const HopArgs &a, int clov, bool xpay, int red, int block, hipStream_t s)
{
    if (!xpay && red == 0) {
        if (clov == 0) return launch_nt<P, NL, DAG, 0, false, 0>(a, block, s);
        if (clov == 2) return launch_nt<P, NL, DAG, 2, false, 0>(a, block, s);
    } else if (xpay) {
        if (clov == 0 && red == 0) return launch_nt<P, NL, DAG, 0, true, 0>(a, block, s);
        if (clov == 0 && red == 1) return launch_nt<P, NL, DAG, 0, true, 1>(a, block, s);
        if (clov == 0 && red == 2) return launch_nt<P, NL, DAG, 0, true, 2>(a, block, s);
        if (clov == 1 && red == 0) return launch_nt<P, NL, DAG, 1, true, 0>(a, block, s);
        if (clov == 1 && red == 1) return launch_nt<P, NL, DAG, 1, true, 1>(a, block, s);
        if (clov == 1 && red == 2) return launch_nt<P, NL, DAG, 1, true, 2>(a, block, s);
        if (clov == 2 && red == 0) return launch_nt<P, NL, DAG, 2, true, 0>(a, block, s);
    }
    return hipErrorInvalidValue;
}

template <int P>
static hipError_t launch_p(const HopArgs &a, int recon, bool dag, int clov, bool xpay, int red, int block,
                           hipStream_t s)
{
    if (recon == 18) {
        return dag ? launch_epi<P, 18, true>(a, clov, xpay, red, block, s)
                   : launch_epi<P, 18, false>(a, clov, xpay, red, block, s);
    }
    if constexpr (P != F64) {
        if (recon == 12)
            return dag ? launch_epi<P, 12, true>(a, clov, xpay, red, block, s)
                       : launch_epi<P, 12, false>(a, clov, xpay, red, block, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lq
