// dslash.h -- the Wilson hopping term of eq. (1) (Sec. 3) on one parity,
// with fused clover / axpy epilogues, for gfx950.
//
// For every output site x of parity p the kernel sums the eight neighbour
// terms of eq. (1):
//     (1 - gamma_mu) U_mu(x) psi(x+mu)  +  (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)
// (signs of gamma swapped for the dagger).  In the chiral basis
// gamma_mu = [[0, B], [B^dag, 0]] with B unitary, so (1 + s gamma_mu) psi is
// fixed by the two upper spin components h = psi_up + s B psi_dn: the lower
// ones are s B^dag h.  Each term is therefore one spin projection to h
// (2 spins x 3 colours), two SU(3) mat-vecs on h, and a reconstruction.
#pragma once

#include "lq_common.h"

namespace lq {

// Epilogue applied to res = coef * (H in), clover mode CLOV = clov & 3:
//   CLOV == 3: res = C res (before the axpy)
//   XPAY:      res = (CLOV == 1 ? C y : y) + res
//   CLOV == 2: res = C res
// where C is the packed clover block field of the output parity (A or A^-1),
// or, with the bit kTwist in clov (clov null), the twisted-mass diagonal
// A = 1 + i tau gamma_5 or its inverse (one right-hand side per thread).
constexpr int kTwist = 4;
struct HopArgs {
    Geom g;
    int p_out;           // output parity
    int nrhs;
    const char *in;      // input field (parity 1 - p_out) base, rhs 0
    long in_n;           // plane stride of the input (sites)
    long in_rs;          // bytes between right-hand sides
    char *out;
    long out_n;
    long out_rs;
    const char *y;       // axpy operand at output sites (same layout as out)
    long y_n;
    long y_rs;
    const char *links;   // packed links [parity][mu] (vh sites each)
    const char *clov;    // packed clover blocks of the output parity (vh sites), or null: then
    double tw_re, tw_im; // the twisted-mass factor on spins 0, 1 (its conjugate on spins 2, 3)
    double coef;
    double *partial;     // per-wavefront partial sums (reduction epilogue) or null
    const char *w;       // second operand of a fused dot product, or null
    long w_n;
    long w_rs;
    int xcd_remap;       // 1: XCD-aware tile order (result independent of it)
    // slice order: > 0 when one time slice of the output parity is exactly
    // slice_tiles workgroups; the tiles of tgroup consecutive slices are then
    // visited slice-fastest (result independent of it)
    int slice_tiles;
    int tgroup;
    // per-rhs freeze mask (solver scalars): a right-hand side r with
    // mask[r * mask_stride + mask_off0] or [.. + mask_off1] nonzero is skipped
    const double *mask;
    int mask_stride, mask_off0, mask_off1;
};

// Launch the hopping kernel.  prec: storage precision; recon: 18 or 12;
// dag: hop with the signs of H^dag; clov: 0 none, 1 on y, 2 on the result,
// 3 on the hopping term before the axpy (with xpay, not with dag);
// xpay: add y; red: 0 none, 2 <w, out>, 3 <w, out> and |out|^2 per
// right-hand side (of the values as stored), written as one partial per
// 64-site wavefront to partial[((rhs * nw) + cb / 64) * K + k], K = 2 or 3,
// nw = ceil(vh / 64); red needs xpay and one right-hand side per thread.
// nr: right-hand sides per thread (1, or 2 without reduction);
// block: threads per workgroup (64, 128 or 256).
hipError_t launch_hop(const HopArgs &a, int prec, int recon, bool dag, int clov, bool xpay, int red, int nr, int block,
                      hipStream_t s);

// The hopping term of up to kMaxBatch lattices in one launch: lattice i's
// arguments a[i] (its geometry, links, clover blocks and field slices, the
// right-hand sides of its systems) and its workgroups tile_off[i] ..
// tile_off[i + 1] - 1 (hop_blocks(vh_i, 64) * ceil(nrhs_i / nr) of them), in
// plain order.  nr = 1: 64 threads per workgroup, one right-hand side per
// thread; nr = 4 (FP16 / FP32): 256 threads, four right-hand sides of a site
// block per workgroup with its links and clover blocks staged in LDS.
constexpr int kMaxBatch = 8;
struct HopBatch {
    HopArgs a[kMaxBatch];
    int tile_off[kMaxBatch + 1];
    int nlat;
    int nr;
};
// (passed by value as the kernel's argument, within the 4 KiB of kernel arguments)
static_assert(sizeof(HopBatch) <= 4096, "HopBatch exceeds the kernel argument space");
hipError_t launch_hop_batch(const HopBatch &b, int prec, int recon, bool dag, int clov, bool xpay, int red,
                            hipStream_t s);

// A tile of the hopping kernel with the neighbour spinors staged in LDS:
// 256 threads, ty * tz * tt whole x-rows (lxh sites each) of the output
// parity, lxh * ty a multiple of 64; ny * nz * nt tiles cover the lattice;
// nrows rows staged (the tile's own and its six faces).
struct HaloTile {
    int ty, tz, tt;
    int ny, nz, nt;
    int nrows;
    int sx, sy, sz;  // log2 of lxh, ty, tz (all powers of two: their product divides 256)
};
// The tile for geometry g, if one fits (lxh * ty * tz * tt == 256, lxh * ty a
// multiple of 64, each extent dividing the lattice; the fewest staged rows).
bool halo_tile(const Geom &g, HaloTile &t);
// LDS bytes of the staged spinors of a tile in precision prec.
inline size_t halo_lds_bytes(int prec, const HaloTile &t, int lxh)
{
    const size_t n = (size_t)t.nrows * lxh;
    return n * (prec == F64 ? 192 : prec == F32 ? 96 : 52);
}
// The hopping term with staged neighbours (one right-hand side; arguments
// and results as launch_hop).
hipError_t launch_hop_halo(const HopArgs &a, const HaloTile &t, int prec, int recon, bool dag, int clov, bool xpay,
                           int red, hipStream_t s);

// Number of workgroups launch_hop uses for a lattice of vh sites.
inline int hop_blocks(int vh, int block) { return (vh + block - 1) / block; }

}  // namespace lq
