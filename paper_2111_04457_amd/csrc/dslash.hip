// dslash.hip -- dispatch of the hopping kernels by storage precision and sign.
#include "dslash.h"

namespace lq {

hipError_t launch_hop_f64_n(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s);
hipError_t launch_hop_f64_d(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s);
hipError_t launch_hop_f32_n(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s);
hipError_t launch_hop_f32_d(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s);
hipError_t launch_hop_f16_n(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s);
hipError_t launch_hop_f16_d(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s);

hipError_t launch_hop_batch_f64_n(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s);
hipError_t launch_hop_batch_f64_d(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s);
hipError_t launch_hop_batch_f32_n(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s);
hipError_t launch_hop_batch_f32_d(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s);
hipError_t launch_hop_batch_f16_n(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s);
hipError_t launch_hop_batch_f16_d(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s);

hipError_t launch_hop_halo_f16_n(const HopArgs &a, const HaloTile &t, int recon, int clov, bool xpay, int red,
                                 hipStream_t s);
hipError_t launch_hop_halo_f16_d(const HopArgs &a, const HaloTile &t, int recon, int clov, bool xpay, int red,
                                 hipStream_t s);

// binary16 only: the staged spinors of a tile take 52 bytes per site in LDS
// (FP32 96, FP64 192: beyond a workgroup's default 64 KiB at these tiles)
hipError_t launch_hop_halo(const HopArgs &a, const HaloTile &t, int prec, int recon, bool dag, int clov, bool xpay,
                           int red, hipStream_t s)
{
    if (prec != F16 || a.nrhs != 1) return hipErrorInvalidValue;
    return dag ? launch_hop_halo_f16_d(a, t, recon, clov, xpay, red, s)
               : launch_hop_halo_f16_n(a, t, recon, clov, xpay, red, s);
}

bool halo_tile(const Geom &g, HaloTile &t)
{
    const int lxh = g.lxh;
    if (lxh < 1 || 256 % lxh != 0) return false;  // lxh, and every tile extent below, a power of two
    const int rows = 256 / lxh;
    bool found = false;
    int best = 0;
    for (int ty = 1; ty <= rows; ++ty) {
        if (rows % ty || g.L[1] % ty || (lxh * ty) % 64) continue;
        for (int tz = 1; tz <= rows / ty; ++tz) {
            if ((rows / ty) % tz || g.L[2] % tz) continue;
            const int tt = rows / (ty * tz);
            if (g.L[3] % tt) continue;
            const int staged = ty * tz * tt + 2 * (tz * tt + ty * tt + ty * tz);
            if (!found || staged < best) {
                found = true;
                best = staged;
                t = HaloTile{ty, tz, tt, g.L[1] / ty, g.L[2] / tz, g.L[3] / tt, staged,
                             __builtin_ctz(lxh), __builtin_ctz(ty), __builtin_ctz(tz)};
            }
        }
    }
    return found;
}

hipError_t launch_hop_batch(const HopBatch &b, int prec, int recon, bool dag, int clov, bool xpay, int red,
                            hipStream_t s)
{
    if (b.nlat < 1 || b.nlat > kMaxBatch) return hipErrorInvalidValue;
    switch (prec) {
    case F64: return dag ? launch_hop_batch_f64_d(b, recon, clov, xpay, red, s)
                         : launch_hop_batch_f64_n(b, recon, clov, xpay, red, s);
    case F32: return dag ? launch_hop_batch_f32_d(b, recon, clov, xpay, red, s)
                         : launch_hop_batch_f32_n(b, recon, clov, xpay, red, s);
    case F16: return dag ? launch_hop_batch_f16_d(b, recon, clov, xpay, red, s)
                         : launch_hop_batch_f16_n(b, recon, clov, xpay, red, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_hop(const HopArgs &a, int prec, int recon, bool dag, int clov, bool xpay, int red, int nr, int block,
                      hipStream_t s)
{
    switch (prec) {
    case F64: return dag ? launch_hop_f64_d(a, recon, clov, xpay, red, nr, block, s)
                         : launch_hop_f64_n(a, recon, clov, xpay, red, nr, block, s);
    case F32: return dag ? launch_hop_f32_d(a, recon, clov, xpay, red, nr, block, s)
                         : launch_hop_f32_n(a, recon, clov, xpay, red, nr, block, s);
    case F16: return dag ? launch_hop_f16_d(a, recon, clov, xpay, red, nr, block, s)
                         : launch_hop_f16_n(a, recon, clov, xpay, red, nr, block, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lq
