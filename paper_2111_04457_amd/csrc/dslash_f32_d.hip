// dslash_f32_d.hip -- instantiations of the hopping kernels, F32 storage,
// signs of H^dag.
#include "dslash_impl.h"

namespace lq {

hipError_t launch_hop_f32_d(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s)
{
    return launch_pd<F32, true>(a, recon, clov, xpay, red, nr, block, s);
}

hipError_t launch_hop_batch_f32_d(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s)
{
    return launch_pd_batch<F32, true>(b, recon, clov, xpay, red, s);
}

}  // namespace lq
