// dslash_f32.hip -- instantiations of the hopping kernels for F32 storage.
#include "dslash_impl.h"

namespace lq {

hipError_t launch_hop_f32(const HopArgs &a, int recon, bool dag, int clov, bool xpay, int red, int block,
                         hipStream_t s)
{
    return launch_p<F32>(a, recon, dag, clov, xpay, red, block, s);
}

}  // namespace lq
