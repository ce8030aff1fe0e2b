// dslash_impl.h -- hopping term of eq. (1) (Sec. 3) on one parity for gfx950.
// One thread per output site and group of NR right-hand sides: each link is
// loaded once per direction and applied to the NR neighbour spinors, and the
// clover block once per site.  Fields are read through the plane layout of
// lq_common.h (16-byte elements, a wavefront reads 1 KiB contiguous per
// load).  Neighbour spinors are re-used through the L2 and the Infinity
// Cache; links are read once per NR right-hand sides.
#pragma once

#include "dslash.h"
#include "stencil.h"

namespace lq {

// The eight neighbour terms are processed as a software pipeline over
// "halves" k = 0..7 (direction k/2, forward for even k): the loads of half
// k + PF are issued before half k is computed, so every thread keeps PF
// neighbours' links and spinors in flight.  The loads land in raw storage
// registers (binary16 data stays packed until it is used).
template <int P, int NL, int NR> struct HalfRaw {
    typename PT<P>::S link[NL];
    typename PT<P>::S sp[NR][24];
    float scale[NR];
    bool wrap;
};

// a b - c d for binary16 operands, as 8 multiply-adds (each reads its
// binary16 operands directly; 14 operations with separate products)
__device__ __forceinline__ cx<float> cdet2(cx<float> a, cx<float> b, cx<float> c, cx<float> d)
{
    const float tr = fmar(-c.im, d.im, mul16(c.re, d.re));
    const float tim = fmar(c.im, d.re, mul16(c.re, d.im));
    return cx<float>{fmar(-a.im, b.im, fmar(a.re, b.re, -tr)), fmar(a.im, b.re, fmar(a.re, b.im, -tim))};
}

// The link of half K of site cb (parity p_out): U_mu(x) forward, U_mu(x - mu) backward.
template <int P, int NL, int K, bool NTL>
__device__ __forceinline__ void load_half_link(const HopArgs &a, int cb, int nb, typename PT<P>::S *link)
{
    using S = typename PT<P>::S;
    constexpr int MU = K / 2;
    if constexpr ((K % 2) == 0)
        load_planes<S, NL, NTL>(a.links + (long)(a.p_out * 4 + MU) * Planes<S, NL>::field_bytes(a.g.vh), cb, a.g.vh,
                                link);
    else
        load_planes<S, NL, NTL>(a.links + (long)((1 - a.p_out) * 4 + MU) * Planes<S, NL>::field_bytes(a.g.vh), nb,
                                a.g.vh, link);
}

// Neighbour index and wrap flag of half K.
template <int K>
__device__ __forceinline__ int half_neighbour(const HopArgs &a, const int c[4], bool &wrap)
{
    constexpr int MU = K / 2;
    int d[4] = {c[0], c[1], c[2], c[3]};
    if constexpr ((K % 2) == 0) {
        wrap = (d[MU] == a.g.L[MU] - 1);
        d[MU] = wrap ? 0 : d[MU] + 1;
    } else {
        wrap = (d[MU] == 0);
        d[MU] = wrap ? a.g.L[MU] - 1 : d[MU] - 1;
    }
    return cb_index(a.g, d);
}

// LINK = false: the link is not loaded (the caller reads it from LDS).
template <int P, int NL, int NR, int K, bool NTL = false, bool LINK = true>
__device__ __forceinline__ void gather(const HopArgs &a, const char *__restrict__ in, int nr, int cb, const int c[4],
                                       HalfRaw<P, NL, NR> &h)
{
    using S = typename PT<P>::S;
    const int nb = half_neighbour<K>(a, c, h.wrap);
    if constexpr (LINK) load_half_link<P, NL, K, NTL>(a, cb, nb, h.link);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        // right-hand sides past the group's end re-read the last one (discarded)
        const int rr = r < nr ? r : nr - 1;
        const char *base = in + rr * a.in_rs;
        load_planes<S, 24>(base, nb, a.in_n, h.sp[r]);
        if constexpr (PT<P>::scaled)
            h.scale[r] = *reinterpret_cast<const float *>(base + 48 * (size_t)padded_sites(a.in_n) + (uint32_t)nb * 4u);
    }
}

// The third row of an SU(3) link from its first two rows (u[0..5] as
// converted from storage): conj(row0 x row1).  Binary16 storage forms it
// with the multiply-adds of cdet2; FP32 / FP64 with the complex products.
// Every kernel that rebuilds a row calls this, so all round alike.
template <int P>
__device__ __forceinline__ void third_row(cx<typename PT<P>::R> u[9])
{
    if constexpr (PT<P>::scaled) {
        u[6] = conj(cdet2(u[1], u[5], u[2], u[4]));
        u[7] = conj(cdet2(u[2], u[3], u[0], u[5]));
        u[8] = conj(cdet2(u[0], u[4], u[1], u[3]));
    } else {
        u[6] = conj(u[1] * u[5] - u[2] * u[4]);
        u[7] = conj(u[2] * u[3] - u[0] * u[5]);
        u[8] = conj(u[0] * u[4] - u[1] * u[3]);
    }
}

// Half K on the link with real and imaginary part of entry j at
// lnk[2 j LS] and lnk[2 j LS + IM] (IM = LS: reals LS apart; IM = 1:
// (re, im) pairs 2 LS apart).
template <int P, int NL, bool DAG, int NR, int K, int LS, int IM = LS>
__device__ __forceinline__ void consume_link(const HopArgs &a, const typename PT<P>::S *lnk,
                                             const HalfRaw<P, NL, NR> &h, cx<typename PT<P>::R> (&acc)[NR][12])
{
    using R = typename PT<P>::R;
    constexpr int MU = K / 2;
    constexpr bool FWD = (K % 2) == 0;
    // forward: (1 - gamma) U(x) for H, (1 + gamma) for H^dag; backward the opposite sign with U(x-mu)^dag
    constexpr int SG = (FWD ? (DAG ? +1 : -1) : (DAG ? -1 : +1));
    cx<R> u[9];
#pragma unroll
    for (int i = 0; i < NL / 2; ++i) u[i] = cx<R>{(R)lnk[(2 * i) * LS], (R)lnk[(2 * i) * LS + IM]};
    const cx<R> ph = cx<R>{(R)a.g.bc_re[MU], FWD ? (R)a.g.bc_im[MU] : -(R)a.g.bc_im[MU]};
    if constexpr (PT<P>::scaled) {
        // binary16 storage (the kernels are bound by instruction issue as much
        // as by memory): the projection is one packed binary16 add per
        // complex component of the stored spinor, the colour product two
        // binary16 dot products per complex multiply-add (FP32 sums), and the
        // spinor's scale is folded into the reconstruction's multiply-adds;
        // the boundary phase (a scalar, so it commutes with U) multiplies the
        // product, only where it is not 1.  The third link row is rebuilt in
        // FP32 from the converted entries and rounded to binary16.
        h2 uh[9];
#pragma unroll
        for (int i = 0; i < NL / 2; ++i) uh[i] = h2{lnk[(2 * i) * LS], lnk[(2 * i) * LS + IM]};
        if constexpr (NL == 12) {
            third_row<P>(u);
#pragma unroll
            for (int i = 6; i < 9; ++i) uh[i] = h2{to_f16(u[i].re), to_f16(u[i].im)};
        }
        const bool phase = a.g.bc_re[MU] != 1.0 || a.g.bc_im[MU] != 0.0;  // the same for every thread
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            h2 ps[12], hh[6], hs[6];
#pragma unroll
            for (int i = 0; i < 12; ++i) ps[i] = h2{h.sp[r][2 * i], h.sp[r][2 * i + 1]};
            cx<R> o[6];
            project_h2<MU, SG>(ps, hh, hs);
            su3_mul_h2<!FWD>(uh, hh, hs, o);
            if (phase && h.wrap) {
#pragma unroll
                for (int i = 0; i < 6; ++i) o[i] = ph * o[i];
            }
            reconstruct_sc<MU, SG>(acc[r], o, h.scale[r]);
        }
    } else {
        if constexpr (NL == 12) third_row<P>(u);
        // FP32 / FP64 are bound by memory: a branch-free multiply by the
        // boundary phase keeps the loads of the pipeline free to move (a
        // branch here measured slower)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            Spinor<R> ps;
#pragma unroll
            for (int i = 0; i < 12; ++i) ps.c[i] = cx<R>{(R)h.sp[r][2 * i], (R)h.sp[r][2 * i + 1]};
            cx<R> hh[6], o[6];
            project<MU, SG>(ps, hh);
            const cx<R> f = h.wrap ? ph : cx<R>{1, 0};
#pragma unroll
            for (int i = 0; i < 6; ++i) hh[i] = f * hh[i];
            su3_mul<!FWD>(u, hh, o);
            reconstruct<MU, SG>(acc[r], o);
        }
    }
}

template <int P, int NL, bool DAG, int NR, int K>
__device__ __forceinline__ void consume(const HopArgs &a, const HalfRaw<P, NL, NR> &h,
                                        cx<typename PT<P>::R> (&acc)[NR][12])
{
    consume_link<P, NL, DAG, NR, K, 1>(a, h.link, h, acc);
}

// Pipeline step K: compute half K from slot K % PF, then refill that slot
// with half K + PF.
template <int P, int NL, bool DAG, int NR, int PF, int K, bool NTL>
__device__ __forceinline__ void pipeline(const HopArgs &a, const char *__restrict__ in, int nr, int cb, const int c[4],
                                         HalfRaw<P, NL, NR> (&slot)[PF], cx<typename PT<P>::R> (&acc)[NR][12])
{
    if constexpr (K < 8) {
        consume<P, NL, DAG, NR, K>(a, slot[K % PF], acc);
        if constexpr (K + PF < 8) gather<P, NL, NR, K + PF, NTL>(a, in, nr, cb, c, slot[K % PF]);
        pipeline<P, NL, DAG, NR, PF, K + 1, NTL>(a, in, nr, cb, c, slot, acc);
    }
}

template <int P, int NL, int NR, int PF, int K, bool NTL>
__device__ __forceinline__ void prologue(const HopArgs &a, const char *__restrict__ in, int nr, int cb, const int c[4],
                                         HalfRaw<P, NL, NR> (&slot)[PF])
{
    if constexpr (K < PF) {
        gather<P, NL, NR, K, NTL>(a, in, nr, cb, c, slot[K]);
        prologue<P, NL, NR, PF, K + 1, NTL>(a, in, nr, cb, c, slot);
    }
}

// Tile k of the visiting order -> site block.  The site blocks of tg
// consecutive time slices (S blocks per slice) are visited slice-fastest:
// the t +- 1 neighbours of a block were read a few workgroups earlier and are
// still in the L2, where in plain order they lie a whole slice of links and
// spinors (more than the L2 holds) away.
__device__ __forceinline__ int slice_order(int k, int S, int tg, int Lt)
{
    const int gsz = tg * S;
    const int grp = k / gsz;
    const int l = k - grp * gsz;
    const int nt = min(tg, Lt - grp * tg);
    const int j = l / nt;
    const int tt = l - j * nt;
    return (grp * tg + tt) * S + j;
}

// prefetch depth (halves in flight per thread) by storage precision
// (several right-hand sides per thread already multiply the loads in flight)
template <int P, int NR> struct Prefetch {
    static constexpr int base = P == F16 ? 4 : P == F32 ? 2 : 1;
    static constexpr int value = base / NR > 0 ? base / NR : 1;
};

// Cache policy: bit 0 non-temporal link loads, bit 1 non-temporal output
// stores.  Links and results are touched once per apply; streaming them past
// the caches keeps the L2 for the neighbour spinors that are read eight
// times.  Measured on the 32^3 x 64 lattice: both bits pay in every kernel
// except the plain binary16 hop, where the non-temporal stores alone are
// fastest, and the binary16 kernel with the clover block on the result (the
// Schur operator's first kernel), whose output -- the next kernel's
// neighbour spinors, 52 B per odd site -- is better kept in the caches
// (1 % faster).  The clover blocks, read once, are always loaded
// non-temporally (FP32 Schur operator 330 -> 307 us, binary16 1 % faster).
template <int P, int CLOV> struct CachePolicy {
    static constexpr int value = (P == F16 && CLOV == 0) ? 2 : (P == F16 && (CLOV & 3) == 2) ? 1 : 3;
};

// The epilogue's site-local factor C is chosen at compile time: the clover
// mode (CLOV & 3: 0 none, 1 on y, 2 on the result, 3 on the hopping term
// before the axpy) and, with bit kTwist, the twisted-mass factor in place of
// a clover block.  A runtime choice between the two costs the FP64 clover
// kernels their register budget (the 72-real block is then loaded under a
// branch, next to the other path's registers).
template <int CLOV> constexpr int clov_mode() { return CLOV & 3; }
template <int CLOV> constexpr bool has_block() { return (CLOV & 3) != 0 && (CLOV & kTwist) == 0; }
// the four-per-workgroup kernel stages the clover block in LDS next to the
// links in binary16 and FP32; the FP64 block (36 KB per 64 sites) is read by
// each wavefront from the caches instead, so that two workgroups fit a CU
template <int P, int CLOV> constexpr bool stage_block() { return has_block<CLOV>() && P != F64; }

// C v: a clover block (A or A^-1, two 6x6 Hermitian blocks, already loaded
// into craw), or, for the twisted-mass Wilson operator, the scalar tw on
// spins 0, 1 and its conjugate on spins 2, 3 (A = 1 + i tau gamma_5 or its
// inverse, conjugated for the dagger).
template <int CLOV, typename S, typename R>
__device__ __forceinline__ void diag_mul(const HopArgs &a, const S *__restrict__ craw, Spinor<R> &v)
{
    if constexpr ((CLOV & kTwist) != 0) {
        const cx<R> c = cx<R>{(R)a.tw_re, (R)a.tw_im};
#pragma unroll
        for (int i = 0; i < 6; ++i) v.c[i] = c * v.c[i];
#pragma unroll
        for (int i = 6; i < 12; ++i) v.c[i] = conj(c) * v.c[i];
    } else {
        clover_mul_raw(craw, v);
    }
}

// The epilogue of one site: res = coef * acc, then the axpy / clover terms,
// the store, and the fused dot products of the values as stored.
template <int P, int CLOV, bool XPAY, int RED, int NR, int CACHE>
__device__ __forceinline__ void epilogue(const HopArgs &a, int cb, int rhs0, int nr, const typename PT<P>::S *craw,
                                         const cx<typename PT<P>::R> (&acc)[NR][12], double (&red0)[NR],
                                         double (&red1)[NR], double (&red2)[NR])
{
    using R = typename PT<P>::R;
    const R coef = (R)a.coef;
    const bool unit = a.coef == 1.0;  // the same for every thread: no multiply by 1
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < nr) {
            const int rhs = rhs0 + r;
            Spinor<R> res;
#pragma unroll
            for (int i = 0; i < 12; ++i) res.c[i] = unit ? acc[r][i] : coef * acc[r][i];
            if constexpr (clov_mode<CLOV>() == 3) diag_mul<CLOV>(a, craw, res);
            if constexpr (XPAY) {
                Spinor<R> yv = load_spinor<P>(a.y + rhs * a.y_rs, cb, a.y_n);
                if constexpr (clov_mode<CLOV>() == 1) diag_mul<CLOV>(a, craw, yv);
#pragma unroll
                for (int i = 0; i < 12; ++i) res.c[i] = yv.c[i] + res.c[i];
            }
            if constexpr (clov_mode<CLOV>() == 2) diag_mul<CLOV>(a, craw, res);
            store_spinor<P, (CACHE & 2) != 0>(a.out + rhs * a.out_rs, cb, a.out_n, res);
            if constexpr (RED != 0) {
                // <w, out> (and |out|^2) of the values as stored
                const Spinor<R> sv = as_stored<P>(res);
                const Spinor<R> wv = load_spinor<P>(a.w + rhs * a.w_rs, cb, a.w_n);
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    const cx<R> q = cmulc(wv.c[i], sv.c[i]);
                    red0[r] += (double)q.re;
                    red1[r] += (double)q.im;
                    if constexpr (RED == 3) red2[r] += (double)norm2(sv.c[i]);
                }
            }
        }
    }
    }

// One partial per wavefront of 64 consecutive sites, indexed by its first
// site (wave = that site / 64): the sums depend neither on the workgroup
// size nor on the order in which workgroups run.
template <int RED, int NR>
__device__ __forceinline__ void write_partials(const HopArgs &a, long wave, int rhs0, int nr, double (&red0)[NR],
                                               double (&red1)[NR], double (&red2)[NR])
{
    constexpr int K = RED == 2 ? 2 : 3;
    const long nw = ((long)a.g.vh + 63) / 64;
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < nr) {
            const double s0 = wave_sum(red0[r]);
            const double s1 = wave_sum(red1[r]);
            const double s2 = RED == 3 ? wave_sum(red2[r]) : 0.0;
            if (lead && wave < nw) {
                double *o = a.partial + ((long)(rhs0 + r) * nw + wave) * K;
                o[0] = s0;
                o[1] = s1;
                if constexpr (K == 3) o[2] = s2;
            }
        }
    }
}

// One workgroup of the hopping term: tile `id` of the launch (site block and
// group of right-hand sides, in the visiting order below).
template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int NT, int NR, int PF = Prefetch<P, NR>::value,
          int CACHE = CachePolicy<P, CLOV>::value>
__device__ __forceinline__ void hop_body(const HopArgs &a, const int id)
{
    using R = typename PT<P>::R;
    using S = typename PT<P>::S;
    // Workgroups are dispatched to the 8 XCDs round-robin; give each XCD a
    // contiguous range of (site block, rhs group) tiles so that neighbour
    // spinors and the links shared by the groups of a site block are
    // re-read from that XCD's L2.  The rhs group varies fastest.
    const int nbs = (a.g.vh + NT - 1) / NT;
    const int ngr = (a.nrhs + NR - 1) / NR;
    const int total = nbs * ngr;
    const int full = a.xcd_remap ? (total / 8) * 8 : 0;
    const int t = id < full ? (id % 8) * (full / 8) + id / 8 : id;
    const int k = t / ngr;
    const int rhs0 = (t - k * ngr) * NR;
    const int sblk = a.slice_tiles > 0 ? slice_order(k, a.slice_tiles, a.tgroup, a.g.L[3]) : k;
    int nr = min(NR, a.nrhs - rhs0);
    // a tile whose right-hand sides are all frozen (converged or broken-down
    // systems of a solver) exits at once; a tile with a live one runs whole
    if (a.mask) {
        bool any = false;
        for (int r = 0; r < nr; ++r) {
            const double *m = a.mask + (long)(rhs0 + r) * a.mask_stride;
            any = any || (m[a.mask_off0] == 0.0 && m[a.mask_off1] == 0.0);
        }
        if (!any) nr = 0;
    }
    const int cb = sblk * NT + threadIdx.x;
    const bool valid = cb < a.g.vh && nr > 0;
    double red0[NR], red1[NR], red2[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) red0[r] = red1[r] = red2[r] = 0.0;
    if (valid) {
        const char *in = a.in + rhs0 * a.in_rs;
        int c[4];
        cb_coords(a.g, a.p_out, cb, c);
        cx<R> acc[NR][12];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int i = 0; i < 12; ++i) acc[r][i] = cx<R>{0, 0};
        HalfRaw<P, NL, NR> slot[PF];
        prologue<P, NL, NR, PF, 0, (CACHE & 1) != 0>(a, in, nr, cb, c, slot);
        pipeline<P, NL, DAG, NR, PF, 0, (CACHE & 1) != 0>(a, in, nr, cb, c, slot, acc);
        S craw[has_block<CLOV>() ? 72 : 1];
        if constexpr (has_block<CLOV>()) load_planes<S, 72, true>(a.clov, cb, a.g.vh, craw);
        epilogue<P, CLOV, XPAY, RED, NR, CACHE>(a, cb, rhs0, nr, craw, acc, red0, red1, red2);
    }
    if constexpr (RED != 0) {
        const long wave = ((long)sblk * NT + (threadIdx.x & ~63)) / 64;
        write_partials<RED, NR>(a, wave, rhs0, nr, red0, red1, red2);
    }
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int NT, int NR>
__global__ __launch_bounds__(NT) void hop_kernel(HopArgs a)
{
    hop_body<P, NL, DAG, CLOV, XPAY, RED, NT, NR>(a, blockIdx.x);
}

// The hopping term of several lattices in one launch (a ragged batch): the
// workgroups tile_off[i] .. tile_off[i + 1] - 1 run lattice i's tiles with
// its arguments (64 sites per workgroup, one right-hand side per thread).
template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED>
__global__ __launch_bounds__(64) void hop_batch_kernel(HopBatch b)
{
    const int t = blockIdx.x;
    int i = 0;
    while (i + 1 < b.nlat && t >= b.tile_off[i + 1]) ++i;
    hop_body<P, NL, DAG, CLOV, XPAY, RED, 64, 1>(b.a[i], t - b.tile_off[i]);
}

// ------------------------------------------------ neighbours staged in LDS --
//
// One workgroup of 256 threads per tile of whole x-rows of the output parity
// (lxh sites each): ty x tz x tt rows, lxh * ty a multiple of 64, so that a
// wavefront covers 64 consecutive sites (its partial sums are those of
// hop_body).  Every input spinor the tile needs -- its own rows (the x
// neighbours) and the six faces of rows around it (the y, z, t neighbours)
// -- is read from memory once into LDS; the eight neighbour terms of each
// site then read their spinors from LDS.  The operations are those of
// hop_body in the same order, so the results are the same bits.

// LDS slot of the staged row at offset (dy, dz, dt) from the tile's origin,
// at most one of them outside the tile: the tile's rows, then the y, z and
// t faces (the -1 face before the +T face).
__device__ __forceinline__ int halo_slot(const HaloTile &h, int dy, int dz, int dt)
{
    const int I = h.ty * h.tz * h.tt;
    if (dy < 0 || dy >= h.ty) return I + (dy < 0 ? 0 : h.tz * h.tt) + dz + h.tz * dt;
    if (dz < 0 || dz >= h.tz) return I + 2 * h.tz * h.tt + (dz < 0 ? 0 : h.ty * h.tt) + dy + h.ty * dt;
    if (dt < 0 || dt >= h.tt)
        return I + 2 * h.tz * h.tt + 2 * h.ty * h.tt + (dt < 0 ? 0 : h.ty * h.tz) + dy + h.ty * dz;
    return dy + h.ty * (dz + h.tz * dt);
}

// The offsets of slot s (the inverse of halo_slot); tile extents are powers
// of two (shifts and masks).
__device__ __forceinline__ void halo_offsets(const HaloTile &h, int s, int &dy, int &dz, int &dt)
{
    const int syz = h.sy + h.sz;
    const int I = 1 << (syz + __builtin_ctz(h.tt));
    if (s < I) {
        dy = s & (h.ty - 1);
        dz = (s >> h.sy) & (h.tz - 1);
        dt = s >> syz;
        return;
    }
    s -= I;
    const int fy = h.tz * h.tt, fz = h.ty * h.tt, ft = h.ty * h.tz;
    if (s < 2 * fy) {
        dy = s < fy ? -1 : h.ty;
        s &= fy - 1;
        dz = s & (h.tz - 1);
        dt = s >> h.sz;
        return;
    }
    s -= 2 * fy;
    if (s < 2 * fz) {
        dz = s < fz ? -1 : h.tz;
        s &= fz - 1;
        dy = s & (h.ty - 1);
        dt = s >> h.sy;
        return;
    }
    s -= 2 * fz;
    dt = s < ft ? -1 : h.tt;
    s &= ft - 1;
    dy = s & (h.ty - 1);
    dz = s >> h.sy;
}

__device__ __forceinline__ int wrap_coord(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// Half K of a site whose neighbour spinor is in LDS at (slot, jn): the link
// from memory (loaded before the staging), the term computed as in hop_body.
template <int P, int NL, bool DAG, int K>
__device__ __forceinline__ void halo_half(const HopArgs &a, const HaloTile &h, const char *smem, int nsites,
                                          int slot, int jn, const typename PT<P>::S *link, bool wrap,
                                          cx<typename PT<P>::R> (&acc)[1][12])
{
    using S = typename PT<P>::S;
    constexpr int K16 = Planes<S, 24>::K16;
    HalfRaw<P, NL, 1> hr;
#pragma unroll
    for (int i = 0; i < NL; ++i) hr.link[i] = link[i];
    const int e = slot * a.g.lxh + jn;
    const u32x4 *lsp = reinterpret_cast<const u32x4 *>(smem);
#pragma unroll
    for (int k = 0; k < K16; ++k) {
        const u32x4 q = lsp[(size_t)k * nsites + e];
        __builtin_memcpy(hr.sp[0] + k * (16 / sizeof(S)), &q, 16);
    }
    if constexpr (PT<P>::scaled)
        hr.scale[0] = reinterpret_cast<const float *>(smem + (size_t)K16 * 16 * nsites)[e];
    hr.wrap = wrap;
    consume<P, NL, DAG, 1, K>(a, hr, acc);
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED>
__global__ __launch_bounds__(256) void hop_halo_kernel(HopArgs a, HaloTile h)
{
    using S = typename PT<P>::S;
    using R = typename PT<P>::R;
    constexpr int CACHE = CachePolicy<P, CLOV>::value;
    constexpr bool NTL = (CACHE & 1) != 0;
    constexpr int K16 = Planes<S, 24>::K16;
    static_assert(Planes<S, 24>::TAIL == 0, "spinor records are whole 16-byte planes");
    extern __shared__ __align__(16) char smem[];
    const int lxh = a.g.lxh;
    const int nsites = h.nrows * lxh;
    // a frozen system (the single right-hand side of a solver) exits at once
    if (a.mask && (a.mask[a.mask_off0] != 0.0 || a.mask[a.mask_off1] != 0.0)) return;
    int tile = blockIdx.x;
    const int y0 = (tile % h.ny) * h.ty;
    tile /= h.ny;
    const int z0 = (tile % h.nz) * h.tz;
    const int t0 = (tile / h.nz) * h.tt;
    // this thread's output site: x-row position j, row (ry, rz, rt) of the tile
    const int j = threadIdx.x & (lxh - 1);
    const int r = threadIdx.x >> h.sx;
    const int ry = r & (h.ty - 1);
    const int rz = (r >> h.sy) & (h.tz - 1);
    const int rt = r >> (h.sy + h.sz);
    int c[4];
    c[1] = y0 + ry;
    c[2] = z0 + rz;
    c[3] = t0 + rt;
    const int px = (c[1] + c[2] + c[3] + a.p_out) & 1;
    c[0] = 2 * j + px;
    const int cb = j + lxh * (c[1] + a.g.L[1] * (c[2] + a.g.L[2] * c[3]));
    // the eight links first (from memory, in flight while the spinors are staged)
    S link[8][NL];
    bool wrap[8];
    {
        int nb;
        nb = half_neighbour<0>(a, c, wrap[0]);
        load_half_link<P, NL, 0, NTL>(a, cb, nb, link[0]);
        nb = half_neighbour<1>(a, c, wrap[1]);
        load_half_link<P, NL, 1, NTL>(a, cb, nb, link[1]);
        nb = half_neighbour<2>(a, c, wrap[2]);
        load_half_link<P, NL, 2, NTL>(a, cb, nb, link[2]);
        nb = half_neighbour<3>(a, c, wrap[3]);
        load_half_link<P, NL, 3, NTL>(a, cb, nb, link[3]);
        nb = half_neighbour<4>(a, c, wrap[4]);
        load_half_link<P, NL, 4, NTL>(a, cb, nb, link[4]);
        nb = half_neighbour<5>(a, c, wrap[5]);
        load_half_link<P, NL, 5, NTL>(a, cb, nb, link[5]);
        nb = half_neighbour<6>(a, c, wrap[6]);
        load_half_link<P, NL, 6, NTL>(a, cb, nb, link[6]);
        nb = half_neighbour<7>(a, c, wrap[7]);
        load_half_link<P, NL, 7, NTL>(a, cb, nb, link[7]);
    }
    // stage the input spinors of the tile's rows and faces
    {
        u32x4 *lsp = reinterpret_cast<u32x4 *>(smem);
        float *lsc = reinterpret_cast<float *>(smem + (size_t)K16 * 16 * nsites);
        for (int e = threadIdx.x; e < nsites; e += 256) {
            const int row = e >> h.sx, jj = e & (lxh - 1);
            int dy, dz, dt;
            halo_offsets(h, row, dy, dz, dt);
            const int y = wrap_coord(y0 + dy, a.g.L[1]), z = wrap_coord(z0 + dz, a.g.L[2]),
                      t = wrap_coord(t0 + dt, a.g.L[3]);
            const long g = jj + (long)lxh * (y + a.g.L[1] * (z + (long)a.g.L[2] * t));
            const char *blk = a.in + (size_t)(g >> 6) * (size_t)(Planes<S, 24>::BYTES * SB);
            const uint32_t lane = (uint32_t)(g & 63);
#pragma unroll
            for (int k = 0; k < K16; ++k) lsp[(size_t)k * nsites + e] = ld<u32x4, false>(blk + k * 16 * SB + lane * 16u);
            if constexpr (PT<P>::scaled)
                lsc[e] = *reinterpret_cast<const float *>(a.in + 48 * (size_t)padded_sites(a.in_n) + (uint32_t)g * 4u);
        }
    }
    __syncthreads();
    cx<R> acc[1][12];
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[0][i] = cx<R>{0, 0};
    const int own = halo_slot(h, ry, rz, rt);
    // x: the same row, the neighbouring position (x + 1 -> (x + 1) / 2, x - 1 -> (x - 1) / 2)
    halo_half<P, NL, DAG, 0>(a, h, smem, nsites, own, j + px == lxh ? 0 : j + px, link[0], wrap[0], acc);
    halo_half<P, NL, DAG, 1>(a, h, smem, nsites, own, j - 1 + px < 0 ? lxh - 1 : j - 1 + px, link[1], wrap[1], acc);
    halo_half<P, NL, DAG, 2>(a, h, smem, nsites, halo_slot(h, ry + 1, rz, rt), j, link[2], wrap[2], acc);
    halo_half<P, NL, DAG, 3>(a, h, smem, nsites, halo_slot(h, ry - 1, rz, rt), j, link[3], wrap[3], acc);
    halo_half<P, NL, DAG, 4>(a, h, smem, nsites, halo_slot(h, ry, rz + 1, rt), j, link[4], wrap[4], acc);
    halo_half<P, NL, DAG, 5>(a, h, smem, nsites, halo_slot(h, ry, rz - 1, rt), j, link[5], wrap[5], acc);
    halo_half<P, NL, DAG, 6>(a, h, smem, nsites, halo_slot(h, ry, rz, rt + 1), j, link[6], wrap[6], acc);
    halo_half<P, NL, DAG, 7>(a, h, smem, nsites, halo_slot(h, ry, rz, rt - 1), j, link[7], wrap[7], acc);
    S craw[has_block<CLOV>() ? 72 : 1];
    if constexpr (has_block<CLOV>()) load_planes<S, 72, true>(a.clov, cb, a.g.vh, craw);
    double red0[1] = {0.0}, red1[1] = {0.0}, red2[1] = {0.0};
    epilogue<P, CLOV, XPAY, RED, 1, CACHE>(a, cb, 0, 1, craw, acc, red0, red1, red2);
    if constexpr (RED != 0) write_partials<RED, 1>(a, cb >> 6, 0, 1, red0, red1, red2);
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED>
static hipError_t launch_halo1(const HopArgs &a, const HaloTile &h, hipStream_t s)
{
    const size_t lds = halo_lds_bytes(P, h, a.g.lxh);
    hop_halo_kernel<P, NL, DAG, CLOV, XPAY, RED><<<dim3(h.ny * h.nz * h.nt), 256, lds, s>>>(a, h);
    return hipGetLastError();
}

// The epilogue combinations of launch_epi for the staged kernel.
template <int P, int NL, bool DAG>
static hipError_t launch_epi_halo(const HopArgs &a, const HaloTile &h, int clov, bool xpay, int red, hipStream_t s)
{
    if (!xpay && red == 0) {
        if (clov == 0) return launch_halo1<P, NL, DAG, 0, false, 0>(a, h, s);
        if (clov == 2) return launch_halo1<P, NL, DAG, 2, false, 0>(a, h, s);
    } else if (xpay) {
        if (clov == 0 && red == 0) return launch_halo1<P, NL, DAG, 0, true, 0>(a, h, s);
        if (clov == 0 && red == 2) return launch_halo1<P, NL, DAG, 0, true, 2>(a, h, s);
        if (clov == 0 && red == 3) return launch_halo1<P, NL, DAG, 0, true, 3>(a, h, s);
        if (clov == 1 && red == 0) return launch_halo1<P, NL, DAG, 1, true, 0>(a, h, s);
        if (clov == 1 && red == 2) return launch_halo1<P, NL, DAG, 1, true, 2>(a, h, s);
        if (clov == 1 && red == 3) return launch_halo1<P, NL, DAG, 1, true, 3>(a, h, s);
        if (clov == 2 && red == 0) return launch_halo1<P, NL, DAG, 2, true, 0>(a, h, s);
        if constexpr (!DAG) {
            if (clov == 3 && red == 0) return launch_halo1<P, NL, DAG, 3, true, 0>(a, h, s);
            if (clov == 3 && red == 2) return launch_halo1<P, NL, DAG, 3, true, 2>(a, h, s);
            if (clov == 3 && red == 3) return launch_halo1<P, NL, DAG, 3, true, 3>(a, h, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int P, bool DAG>
static hipError_t launch_pd_halo(const HopArgs &a, const HaloTile &h, int recon, int clov, bool xpay, int red,
                                 hipStream_t s)
{
    if (recon == 18) return launch_epi_halo<P, 18, DAG>(a, h, clov, xpay, red, s);
    if (recon == 12) return launch_epi_halo<P, 12, DAG>(a, h, clov, xpay, red, s);
    return hipErrorInvalidValue;
}

// ------------------------------------------- right-hand sides sharing LDS --
//
// Several right-hand sides per workgroup: 64 sites x R right-hand sides, one
// wavefront per right-hand side.  The waves load the eight links of the 64
// sites (the directions split between them) and the sites' clover blocks
// into LDS once; every wave then runs the pipeline of hop_body on its own
// right-hand side's neighbour spinors, with the links read from LDS.  The
// operations are those of hop_body, so the results are the same bits; the
// links and clover blocks are read from memory once per R right-hand sides.

// Links of NL reals are staged as 18: the third row of a 12-real link is
// rebuilt once here (third_row, rounded to the storage type as the hop
// kernels round it) instead of by every wavefront that reads it.
template <int P, int NL, int K, int R, bool NTL>
__device__ __forceinline__ void stage_links(const HopArgs &a, int w, int lane, int cb, const int c[4],
                                            typename PT<P>::S (*lk)[9][64][2])
{
    using S = typename PT<P>::S;
    using Rt = typename PT<P>::R;
    if constexpr (K < 8) {
        if (K % R == w) {
            bool wrap;
            const int nb = half_neighbour<K>(a, c, wrap);
            S raw[NL];
            load_half_link<P, NL, K, NTL>(a, cb, nb, raw);
#pragma unroll
            for (int i = 0; i < NL; ++i) lk[K][i / 2][lane][i % 2] = raw[i];
            if constexpr (NL == 12) {
                cx<Rt> u[9];
#pragma unroll
                for (int i = 0; i < 6; ++i) u[i] = cx<Rt>{(Rt)raw[2 * i], (Rt)raw[2 * i + 1]};
                third_row<P>(u);
#pragma unroll
                for (int i = 6; i < 9; ++i) {
                    // rounded as consume_link rounds it: to FP32, then to
                    // the storage type (to_f16 keeps the compiler from
                    // fusing the last multiply-add with the conversion)
                    if constexpr (PT<P>::scaled) {
                        lk[K][i][lane][0] = to_f16(u[i].re);
                        lk[K][i][lane][1] = to_f16(u[i].im);
                    } else {
                        lk[K][i][lane][0] = (S)u[i].re;
                        lk[K][i][lane][1] = (S)u[i].im;
                    }
                }
            }
        }
        stage_links<P, NL, K + 1, R, NTL>(a, w, lane, cb, c, lk);
    }
}

template <int P, int PF, int K>
__device__ __forceinline__ void prologue_sp(const HopArgs &a, const char *__restrict__ in, int cb, const int c[4],
                                            HalfRaw<P, 18, 1> (&slot)[PF])
{
    if constexpr (K < PF) {
        gather<P, 18, 1, K, false, false>(a, in, 1, cb, c, slot[K]);
        prologue_sp<P, PF, K + 1>(a, in, cb, c, slot);
    }
}

// (links read from LDS as 18 reals, whatever the storage format)
template <int P, bool DAG, int PF, int K>
__device__ __forceinline__ void pipeline_sp(const HopArgs &a, const char *__restrict__ in, int lane, int cb,
                                            const int c[4], typename PT<P>::S (*lk)[9][64][2],
                                            HalfRaw<P, 18, 1> (&slot)[PF], cx<typename PT<P>::R> (&acc)[1][12])
{
    if constexpr (K < 8) {
        consume_link<P, 18, DAG, 1, K, 64, 1>(a, &lk[K][0][lane][0], slot[K % PF], acc);
        if constexpr (K + PF < 8) gather<P, 18, 1, K + PF, false, false>(a, in, 1, cb, c, slot[K % PF]);
        pipeline_sp<P, DAG, PF, K + 1>(a, in, lane, cb, c, lk, slot, acc);
    }
}

// One workgroup (tile `id`: a site block of 64 and a group of R right-hand
// sides) with the links and clover blocks in the LDS arrays lk and lc.
template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int R, int PF = Prefetch<P, 1>::value,
          int CACHE = CachePolicy<P, CLOV>::value>
__device__ __forceinline__ void hop_shared_body(const HopArgs &a, const int id, typename PT<P>::S (*lk)[9][64][2],
                                                typename PT<P>::S (*lc)[64][2])
{
    using Rt = typename PT<P>::R;
    using S = typename PT<P>::S;
    // tiles (site block of 64, group of R right-hand sides), XCD-aware as in hop_body
    const int nbs = (a.g.vh + 63) / 64;
    const int ngr = (a.nrhs + R - 1) / R;
    const int total = nbs * ngr;
    const int full = a.xcd_remap ? (total / 8) * 8 : 0;
    const int t = id < full ? (id % 8) * (full / 8) + id / 8 : id;
    const int kt = t / ngr;
    const int rhs0 = (t - kt * ngr) * R;
    // site block, in the slice order where it applies (64-site tiles)
    const int k = a.slice_tiles > 0 ? slice_order(kt, a.slice_tiles, a.tgroup, a.g.L[3]) : kt;
    const int nrg = min(R, a.nrhs - rhs0);
    // a group whose right-hand sides are all frozen exits at once (uniformly)
    if (a.mask) {
        bool any = false;
        for (int r = 0; r < nrg; ++r) {
            const double *m = a.mask + (long)(rhs0 + r) * a.mask_stride;
            any = any || (m[a.mask_off0] == 0.0 && m[a.mask_off1] == 0.0);
        }
        if (!any) return;
    }
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int cb = k * 64 + lane;
    const bool site_ok = cb < a.g.vh;
    const bool rhs_ok = w < nrg;
    const int rhs = rhs0 + w;
    int c[4] = {0, 0, 0, 0};
    if (site_ok) cb_coords(a.g, a.p_out, cb, c);
    const char *in = a.in + (long)(rhs_ok ? rhs : rhs0) * a.in_rs;
    HalfRaw<P, 18, 1> slot[PF];  // spinors only (the links come from LDS)
    // the first neighbour spinors are requested before the staging barrier
    if (site_ok && rhs_ok) prologue_sp<P, PF, 0>(a, in, cb, c, slot);
    if (site_ok) {
        stage_links<P, NL, 0, R, (CACHE & 1) != 0>(a, w, lane, cb, c, lk);
        if constexpr (stage_block<P, CLOV>()) {
            if (w == R - 1) {
                S raw[72];
                load_planes<S, 72, true>(a.clov, cb, a.g.vh, raw);
#pragma unroll
                for (int i = 0; i < 72; ++i) lc[i / 2][lane][i % 2] = raw[i];
            }
        }
    }
    __syncthreads();
    double red0[1] = {0.0}, red1[1] = {0.0}, red2[1] = {0.0};
    if (site_ok && rhs_ok) {
        cx<Rt> acc[1][12];
#pragma unroll
        for (int i = 0; i < 12; ++i) acc[0][i] = cx<Rt>{0, 0};
        pipeline_sp<P, DAG, PF, 0>(a, in, lane, cb, c, lk, slot, acc);
        S craw[has_block<CLOV>() ? 72 : 1];
        if constexpr (stage_block<P, CLOV>()) {
#pragma unroll
            for (int i = 0; i < 72; ++i) craw[i] = lc[i / 2][lane][i % 2];
        } else if constexpr (has_block<CLOV>()) {
            load_planes<S, 72, true>(a.clov, cb, a.g.vh, craw);
        }
        epilogue<P, CLOV, XPAY, RED, 1, CACHE>(a, cb, rhs, 1, craw, acc, red0, red1, red2);
    }
    if constexpr (RED != 0) {
        if (rhs_ok) write_partials<RED, 1>(a, k, rhs, 1, red0, red1, red2);
    }
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int R>
__global__ __launch_bounds__(64 * R) void hop_shared_kernel(HopArgs a)
{
    using S = typename PT<P>::S;
    __shared__ S lk[8][9][64][2];
    __shared__ S lc[stage_block<P, CLOV>() ? 36 : 1][64][2];
    hop_shared_body<P, NL, DAG, CLOV, XPAY, RED, R>(a, blockIdx.x, lk, lc);
}

// The same for a ragged batch: the workgroups tile_off[i] .. tile_off[i + 1] - 1
// run lattice i's tiles (groups of R right-hand sides).
template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int R>
__global__ __launch_bounds__(64 * R) void hop_shared_batch_kernel(HopBatch b)
{
    using S = typename PT<P>::S;
    __shared__ S lk[8][9][64][2];
    __shared__ S lc[stage_block<P, CLOV>() ? 36 : 1][64][2];
    const int t = blockIdx.x;
    int i = 0;
    while (i + 1 < b.nlat && t >= b.tile_off[i + 1]) ++i;
    hop_shared_body<P, NL, DAG, CLOV, XPAY, RED, R>(b.a[i], t - b.tile_off[i], lk, lc);
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int R>
static hipError_t launch_shared(const HopArgs &a, hipStream_t s)
{
    const int ngr = (a.nrhs + R - 1) / R;
    const dim3 grid(hop_blocks(a.g.vh, 64) * ngr);
    hop_shared_kernel<P, NL, DAG, CLOV, XPAY, RED, R><<<grid, 64 * R, 0, s>>>(a);
    return hipGetLastError();
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED, int NR>
static hipError_t launch_nt(const HopArgs &a, int block, hipStream_t s)
{
    const int ngr = (a.nrhs + NR - 1) / NR;
    const dim3 grid(hop_blocks(a.g.vh, block) * ngr);
    switch (block) {
    case 64: hop_kernel<P, NL, DAG, CLOV, XPAY, RED, 64, NR><<<grid, 64, 0, s>>>(a); break;
    case 128: hop_kernel<P, NL, DAG, CLOV, XPAY, RED, 128, NR><<<grid, 128, 0, s>>>(a); break;
    case 256: hop_kernel<P, NL, DAG, CLOV, XPAY, RED, 256, NR><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Right-hand sides per thread: NR = 1, or 2 for the epilogues of the
// operators (plain, clover on the result, clover on y with axpy, axpy).
template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED>
static hipError_t launch_nr(const HopArgs &a, int nr, int block, hipStream_t s)
{
    // nr == 4: four right-hand sides per workgroup sharing links in LDS
    if (nr == 4) return launch_shared<P, NL, DAG, CLOV, XPAY, RED, 4>(a, s);
    if constexpr (RED == 0) {
        if (nr == 2) return launch_nt<P, NL, DAG, CLOV, XPAY, RED, 2>(a, block, s);
    }
    if (nr == 1) return launch_nt<P, NL, DAG, CLOV, XPAY, RED, 1>(a, block, s);
    return hipErrorInvalidValue;
}

// The epilogue combinations the operators use:
//   (clov, xpay, red) in {(0,0,0) plain hop, (2,0,0) C H x, (1,1,*) C y + c H x,
//                         (0,1,*) y + c H x, (2,1,0) C (y + c H x), (3,1,*) y + C (c H x)}
// The twisted-mass epilogues (clov | kTwist).
template <int P, int NL, bool DAG>
static hipError_t launch_epi_tw(const HopArgs &a, int clov, bool xpay, int red, int nr, int block, hipStream_t s)
{
    constexpr int T = kTwist;
    if (!xpay && red == 0 && clov == 2) return launch_nr<P, NL, DAG, T | 2, false, 0>(a, nr, block, s);
    if (xpay) {
        if (clov == 1 && red == 0) return launch_nr<P, NL, DAG, T | 1, true, 0>(a, nr, block, s);
        if (clov == 1 && red == 2) return launch_nr<P, NL, DAG, T | 1, true, 2>(a, nr, block, s);
        if (clov == 1 && red == 3) return launch_nr<P, NL, DAG, T | 1, true, 3>(a, nr, block, s);
        if (clov == 2 && red == 0) return launch_nr<P, NL, DAG, T | 2, true, 0>(a, nr, block, s);
        if constexpr (!DAG) {
            if (clov == 3 && red == 0) return launch_nr<P, NL, DAG, T | 3, true, 0>(a, nr, block, s);
            if (clov == 3 && red == 2) return launch_nr<P, NL, DAG, T | 3, true, 2>(a, nr, block, s);
            if (clov == 3 && red == 3) return launch_nr<P, NL, DAG, T | 3, true, 3>(a, nr, block, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int P, int NL, bool DAG>
static hipError_t launch_epi(const HopArgs &a, int clov, bool xpay, int red, int nr, int block, hipStream_t s)
{
    if (clov & kTwist) return launch_epi_tw<P, NL, DAG>(a, clov & 3, xpay, red, nr, block, s);
    if (!xpay && red == 0) {
        if (clov == 0) return launch_nr<P, NL, DAG, 0, false, 0>(a, nr, block, s);
        if (clov == 2) return launch_nr<P, NL, DAG, 2, false, 0>(a, nr, block, s);
    } else if (xpay) {
        if (clov == 0 && red == 0) return launch_nr<P, NL, DAG, 0, true, 0>(a, nr, block, s);
        if (clov == 0 && red == 2) return launch_nr<P, NL, DAG, 0, true, 2>(a, nr, block, s);
        if (clov == 0 && red == 3) return launch_nr<P, NL, DAG, 0, true, 3>(a, nr, block, s);
        if (clov == 1 && red == 0) return launch_nr<P, NL, DAG, 1, true, 0>(a, nr, block, s);
        if (clov == 1 && red == 2) return launch_nr<P, NL, DAG, 1, true, 2>(a, nr, block, s);
        if (clov == 1 && red == 3) return launch_nr<P, NL, DAG, 1, true, 3>(a, nr, block, s);
        if (clov == 2 && red == 0) return launch_nr<P, NL, DAG, 2, true, 0>(a, nr, block, s);
        // y + C (c H x): the A_ee^-1-preconditioned Schur operator (no dagger form)
        if constexpr (!DAG) {
            if (clov == 3 && red == 0) return launch_nr<P, NL, DAG, 3, true, 0>(a, nr, block, s);
            if (clov == 3 && red == 2) return launch_nr<P, NL, DAG, 3, true, 2>(a, nr, block, s);
            if (clov == 3 && red == 3) return launch_nr<P, NL, DAG, 3, true, 3>(a, nr, block, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int P, int NL, bool DAG, int CLOV, bool XPAY, int RED>
static hipError_t launch_batch1(const HopBatch &b, hipStream_t s)
{
    if constexpr (P != F64) {
        if (b.nr == 4) {
            hop_shared_batch_kernel<P, NL, DAG, CLOV, XPAY, RED, 4><<<dim3(b.tile_off[b.nlat]), 256, 0, s>>>(b);
            return hipGetLastError();
        }
    }
    if (b.nr != 1) return hipErrorInvalidValue;
    hop_batch_kernel<P, NL, DAG, CLOV, XPAY, RED><<<dim3(b.tile_off[b.nlat]), 64, 0, s>>>(b);
    return hipGetLastError();
}

// The epilogue combinations of launch_epi for a batch.
template <int P, int NL, bool DAG>
static hipError_t launch_epi_batch(const HopBatch &b, int clov, bool xpay, int red, hipStream_t s)
{
    if (clov & kTwist) {
        constexpr int T = kTwist;
        clov &= 3;
        if (!xpay && red == 0 && clov == 2) return launch_batch1<P, NL, DAG, T | 2, false, 0>(b, s);
        if (xpay) {
            if (clov == 1 && red == 0) return launch_batch1<P, NL, DAG, T | 1, true, 0>(b, s);
            if (clov == 1 && red == 2) return launch_batch1<P, NL, DAG, T | 1, true, 2>(b, s);
            if (clov == 1 && red == 3) return launch_batch1<P, NL, DAG, T | 1, true, 3>(b, s);
            if constexpr (!DAG) {
                if (clov == 3 && red == 0) return launch_batch1<P, NL, DAG, T | 3, true, 0>(b, s);
                if (clov == 3 && red == 2) return launch_batch1<P, NL, DAG, T | 3, true, 2>(b, s);
                if (clov == 3 && red == 3) return launch_batch1<P, NL, DAG, T | 3, true, 3>(b, s);
            }
        }
        return hipErrorInvalidValue;
    }
    if (!xpay && red == 0) {
        if (clov == 0) return launch_batch1<P, NL, DAG, 0, false, 0>(b, s);
        if (clov == 2) return launch_batch1<P, NL, DAG, 2, false, 0>(b, s);
    } else if (xpay) {
        if (clov == 0 && red == 0) return launch_batch1<P, NL, DAG, 0, true, 0>(b, s);
        if (clov == 0 && red == 2) return launch_batch1<P, NL, DAG, 0, true, 2>(b, s);
        if (clov == 0 && red == 3) return launch_batch1<P, NL, DAG, 0, true, 3>(b, s);
        if (clov == 1 && red == 0) return launch_batch1<P, NL, DAG, 1, true, 0>(b, s);
        if (clov == 1 && red == 2) return launch_batch1<P, NL, DAG, 1, true, 2>(b, s);
        if (clov == 1 && red == 3) return launch_batch1<P, NL, DAG, 1, true, 3>(b, s);
        if (clov == 2 && red == 0) return launch_batch1<P, NL, DAG, 2, true, 0>(b, s);
        if constexpr (!DAG) {
            if (clov == 3 && red == 0) return launch_batch1<P, NL, DAG, 3, true, 0>(b, s);
            if (clov == 3 && red == 2) return launch_batch1<P, NL, DAG, 3, true, 2>(b, s);
            if (clov == 3 && red == 3) return launch_batch1<P, NL, DAG, 3, true, 3>(b, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int P, bool DAG>
static hipError_t launch_pd_batch(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s)
{
    if (recon == 18) return launch_epi_batch<P, 18, DAG>(b, clov, xpay, red, s);
    if (recon == 12) return launch_epi_batch<P, 12, DAG>(b, clov, xpay, red, s);
    return hipErrorInvalidValue;
}

template <int P, bool DAG>
static hipError_t launch_pd(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block, hipStream_t s)
{
    if (recon == 18) return launch_epi<P, 18, DAG>(a, clov, xpay, red, nr, block, s);
    if (recon == 12) return launch_epi<P, 12, DAG>(a, clov, xpay, red, nr, block, s);
    return hipErrorInvalidValue;
}

}  // namespace lq
