// dslash_f64_n.hip -- instantiations of the hopping kernels, F64 storage,
// signs of H.
#include "dslash_impl.h"

namespace lq {

hipError_t launch_hop_f64_n(const HopArgs &a, int recon, int clov, bool xpay, int red, int nr, int block,
                         hipStream_t s)
{
    return launch_pd<F64, false>(a, recon, clov, xpay, red, nr, block, s);
}

hipError_t launch_hop_batch_f64_n(const HopBatch &b, int recon, int clov, bool xpay, int red, hipStream_t s)
{
    return launch_pd_batch<F64, false>(b, recon, clov, xpay, red, s);
}

}  // namespace lq
