// dslash_f32_n.hip -- instantiations of the hopping kernels, F32 storage,
// signs of H.
#include "dslash_impl.h"

namespace lq {

hipError_t launch_hop_f32_n(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s)
{
    return launch_pd<F32, false>(a, recon, clov, xpay, red, nr, block, s);
}

hipError_t launch_hop_batch_f32_n(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s)
{
    return launch_pd_batch<F32, false>(b, recon, clov, xpay, red, s);
}

}  // namespace lq
