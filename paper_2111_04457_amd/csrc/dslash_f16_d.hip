// dslash_f16_d.hip -- instantiations of the hopping kernels, F16 storage,
// signs of H^dag.
#include "dslash_impl.h"

namespace lq {

hipError_t launch_hop_f16_d(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s)
{
    return launch_pd<F16, true>(a, recon, clov, xpay, red, nr, block, s);
}

hipError_t launch_hop_batch_f16_d(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s)
{
    return launch_pd_batch<F16, true>(b, recon, clov, xpay, red, s);
}

hipError_t launch_hop_halo_f16_d(const HopArgs &a, const HaloTile &t, int recon, int clov, bool xpay, int red,
                              hipStream_t s)
{
    return launch_pd_halo<F16, true>(a, t, recon, clov, xpay, red, s);
}

}  // namespace lq
