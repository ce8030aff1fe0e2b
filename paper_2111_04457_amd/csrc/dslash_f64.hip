// dslash_f64.hip -- instantiations of the hopping kernels for F64 storage.
#include "dslash_impl.h"

namespace lq {

hipError_t launch_hop_f64(const HopArgs &a, int recon, bool dag, int clov, bool xpay, int red, int block,
                         hipStream_t s)
{
    return launch_p<F64>(a, recon, dag, clov, xpay, red, block, s);
}

}  // namespace lq
