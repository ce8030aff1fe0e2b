// probe.hip -- device bandwidth probes (lq_bandwidth_probe): a plain copy
// and a read-only stream over device buffers, the reference points for the
// HBM roofline of the operator kernels and for scaling the hardware counters.
#include <algorithm>

#include "runtime.h"

namespace lq {

namespace {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int PT_THREADS = 256;

// dst = src, 16 bytes per thread per step, grid-stride, streamed past the caches
__global__ __launch_bounds__(PT_THREADS) void copy_probe_kernel(u4 *__restrict__ dst, const u4 *__restrict__ src,
                                                                 long n)
{
    const long stride = (long)gridDim.x * PT_THREADS;
    for (long i = (long)blockIdx.x * PT_THREADS + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// reads every 16-byte element once; one xor-sum per workgroup to out (so
// that the loads are not dropped)
__global__ __launch_bounds__(PT_THREADS) void read_probe_kernel(const u4 *__restrict__ src, long n,
                                                                 unsigned *__restrict__ out)
{
    const long stride = (long)gridDim.x * PT_THREADS;
    unsigned acc = 0;
    for (long i = (long)blockIdx.x * PT_THREADS + threadIdx.x; i < n; i += stride) {
        const u4 v = __builtin_nontemporal_load(src + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    __shared__ unsigned lds[PT_THREADS];
    lds[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned a = 0;
        for (int k = 0; k < PT_THREADS; ++k) a ^= lds[k];
        out[blockIdx.x] = a;
    }
}

}  // namespace

}  // namespace lq

using namespace lq;

extern "C" lq_status lq_bandwidth_probe(int mode, void *dst, const void *src, size_t bytes, int reps, double *us,
                                        void *stream)
{
    if (!src || !us || (mode == 0 && !dst) || (mode != 0 && mode != 1) || reps < 1) {
        set_error("lq_bandwidth_probe: null argument, unknown mode or reps < 1");
        return LQ_ERR_ARG;
    }
    if (bytes < 16 || (bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15) ||
        (dst && (reinterpret_cast<uintptr_t>(dst) & 15))) {
        set_error("lq_bandwidth_probe: bytes must be a multiple of 16 (>= 16) and the buffers 16-byte aligned");
        return LQ_ERR_ARG;
    }
    try {
        set_error("");
        hipStream_t s = static_cast<hipStream_t>(stream);
        int dev = 0, ncu = 0;
        LQ_HIP(hipGetDevice(&dev));
        LQ_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        const long n = (long)(bytes / 16);
        // enough workgroups for every compute unit, each streaming many elements
        const int grid = (int)std::min<long>((long)std::max(ncu, 1) * 16, (n + PT_THREADS - 1) / PT_THREADS);
        Buf partial;
        if (mode == 1) partial.ensure(sizeof(unsigned) * grid);
        hipEvent_t e0, e1;
        LQ_HIP(hipEventCreate(&e0));
        LQ_HIP(hipEventCreate(&e1));
        auto launch = [&]() {
            if (mode == 0)
                copy_probe_kernel<<<grid, PT_THREADS, 0, s>>>(static_cast<u4 *>(dst), static_cast<const u4 *>(src), n);
            else
                read_probe_kernel<<<grid, PT_THREADS, 0, s>>>(static_cast<const u4 *>(src), n,
                                                              reinterpret_cast<unsigned *>(partial.ptr));
            return hipGetLastError();
        };
        hipError_t e = launch();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        LQ_HIP(e);
        *us = 1e3 * (double)ms / reps;
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}
