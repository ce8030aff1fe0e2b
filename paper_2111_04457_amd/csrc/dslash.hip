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
