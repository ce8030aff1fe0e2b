// dslash.hip -- dispatch of the hopping kernels by storage precision.
#include "dslash.h"

namespace lq {

hipError_t launch_hop_f64(const HopArgs &a, int recon, bool dag, int clov, bool xpay, int red, int block, hipStream_t s);
hipError_t launch_hop_f32(const HopArgs &a, int recon, bool dag, int clov, bool xpay, int red, int block, hipStream_t s);
hipError_t launch_hop_f16(const HopArgs &a, int recon, bool dag, int clov, bool xpay, int red, int block, hipStream_t s);

hipError_t launch_hop(const HopArgs &a, int prec, int recon, bool dag, int clov, bool xpay, int red, int block,
                      hipStream_t s)
{
    switch (prec) {
    case F64: return launch_hop_f64(a, recon, dag, clov, xpay, red, block, s);
    case F32: return launch_hop_f32(a, recon, dag, clov, xpay, red, block, s);
    case F16: return launch_hop_f16(a, recon, dag, clov, xpay, red, block, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lq
