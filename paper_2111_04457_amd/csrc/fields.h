// fields.h -- import/export of spinor and gauge fields between the
// boundary layout (complex128, lexicographic or checkerboard AoS) and the
// packed plane layout, and the clover term A = 1 + F of eq. (1) (Sec. 3).
#pragma once

#include "lq_common.h"

namespace lq {

// One workgroup's share of a ragged field (slices of different lengths, as
// in a batch of lattices): sites blk * 256 .. of slice `slice`, which holds
// n sites and starts site_off padded sites after the field's base.
struct Tile {
    int slice;
    int blk;
    int n;
    int site_off;
};

// A packed spinor field in HBM: nrhs slices of one parity field each,
// `rs` bytes apart, plane stride n sites.  A ragged field (tiles != null)
// holds nrhs slices of their own lengths, back to back; its vector kernels
// run one workgroup per entry of the device array tiles[ntiles] (slice by
// slice, in order).
struct FieldView {
    char *base;
    int prec;
    long n;
    long rs;
    int nrhs;
    const Tile *tiles = nullptr;
    int ntiles = 0;
};

// Spinor import/export.  mode 0: src/dst is a full lexicographic field
// [nrhs][V][4][3] and the view holds parity `p`; mode 1: a parity field
// [nrhs][V/2][4][3] in checkerboard order.
hipError_t launch_pack_spinor(const Geom &g, int p, int mode, const double *src, FieldView dst, hipStream_t s);
hipError_t launch_unpack_spinor(const Geom &g, int p, int mode, FieldView src, double *dst, hipStream_t s);

// Links: U complex128 [V][4][3][3] (lex) -> packed FP64 links [parity][mu]
// (18 reals, row-major, vh sites each).
hipError_t launch_pack_links_f64(const Geom &g, const double *U, char *links64, hipStream_t s);
// FP64 packed links -> packed links of precision prec with nl = 18 or 12
// reals (12: rows 0 and 1).
hipError_t launch_convert_links(const Geom &g, const char *links64, int prec, int nl, char *dst, hipStream_t s);

// Clover blocks A = 1 + F in FP64 (72 reals per site: two packed 6x6
// Hermitian blocks) for both parities, [parity][planes over vh], built from
// the packed FP64 links; fbuf is scratch of clover_fbuf_bytes(vh) bytes
// (the six field strengths of every site).
hipError_t launch_clover_build(const Geom &g, const char *links64, double csw, double kappa, int traceless,
                               char *fbuf, char *clov64, hipStream_t s);
inline size_t clover_fbuf_bytes(long vh) { return (size_t)2 * 6 * 18 * 8 * padded_sites(vh); }
// Per-block inverse of the blocks of parity p by Gauss-Jordan with partial
// pivoting (FP64), into parity p of inv64; sets *flag nonzero if a block is
// singular.
hipError_t launch_clover_invert(const Geom &g, int p, const char *clov64, char *inv64, int *flag, hipStream_t s);
// FP64 packed clover field -> precision prec, parities p0 .. p0 + np - 1.
hipError_t launch_convert_clover(const Geom &g, const char *clov64, int prec, char *dst, hipStream_t s, int p0 = 0,
                                 int np = 2);
// Site-local y = C x on one parity with packed clover C of that parity.
hipError_t launch_clover_apply(const Geom &g, const char *clov, FieldView out, FieldView in, hipStream_t s);
// Site-local y = (c on spins 0, 1, conj(c) on spins 2, 3) x: the twisted-mass
// diagonal 1 + i tau gamma_5 or its inverse.
hipError_t launch_twist_apply(const Geom &g, double c_re, double c_im, FieldView out, FieldView in, hipStream_t s);

__host__ __device__ inline long link_bytes(int prec, int nl, long vh)
{
    return (long)nl * (prec == F64 ? 8 : prec == F32 ? 4 : 2) * padded_sites(vh);
}
__host__ __device__ inline long clover_bytes(int prec, long vh) { return 72L * (prec == F64 ? 8 : prec == F32 ? 4 : 2) * padded_sites(vh); }

}  // namespace lq
