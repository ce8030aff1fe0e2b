// lq_common.h -- device-side building blocks shared by the HIP kernels:
// geometry of the checkerboarded lattice, precision traits, complex
// arithmetic, and loads/stores of the structure-of-arrays field layout.
//
// Field layout in HBM (site blocks of "planes"): the sites of a field are
// grouped in blocks of SB = 64 consecutive sites (one wavefront; the site
// count is padded to whole blocks).  Within a block, a field of R reals per
// site and storage type T is stored as  floor(R*sizeof(T)/16)  planes of
// 16-byte elements, followed by at most one narrower tail plane (8 or 4
// bytes) for the remainder, each plane holding one element per site:
//     plane k element of site s at  base + (s/SB)*REC*SB + k*16*SB + 16*(s%SB)
//     tail element of site s    at  base + (s/SB)*REC*SB + K16*16*SB + TAIL*(s%SB)
// with REC = R*sizeof(T) the bytes of one site.  A wavefront of 64
// consecutive sites reads 64 consecutive 16-byte elements (1 KiB) per load
// instruction, and its whole record is one contiguous range of REC*64 bytes
// (fewer DRAM pages open at a time than with whole-field planes).  FP16
// spinors carry a separate plane of FP32 per-site scales after the blocks.
// Several right-hand sides are stacked whole.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lq {

// ------------------------------------------------------------ precision --

enum Prec { F64 = 0, F32 = 1, F16 = 2 };

template <int P> struct PT;
template <> struct PT<F64> { using S = double;   using R = double; static constexpr bool scaled = false; };
template <> struct PT<F32> { using S = float;    using R = float;  static constexpr bool scaled = false; };
template <> struct PT<F16> { using S = _Float16; using R = float;  static constexpr bool scaled = true; };

// bytes of one site of a field of `reals` reals in storage precision p
__host__ __device__ constexpr long site_bytes(int p, int reals)
{
    return (long)reals * (p == F64 ? 8 : p == F32 ? 4 : 2) + (p == F16 && reals == 24 ? 4 : 0);
}

// ------------------------------------------------------------- complex ---

template <typename R> struct cx {
    R re, im;
};
template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
// All code is compiled without implicit multiply-add contraction; fused
// multiply-adds are written out, so every instantiation of a kernel (any
// launch shape, any number of right-hand sides per thread) rounds exactly
// the same operations and produces bit-identical results.
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// (a plain product: a fused form here doubles the register use of the
// binary16 hopping kernels)
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a b
template <typename R> __device__ __forceinline__ cx<R> cmac(cx<R> acc, cx<R> a, cx<R> b)
{
    return {fmar(a.re, b.re, fmar(-a.im, b.im, acc.re)), fmar(a.re, b.im, fmar(a.im, b.re, acc.im))};
}
// acc + conj(a) b
template <typename R> __device__ __forceinline__ cx<R> cmacc(cx<R> acc, cx<R> a, cx<R> b)
{
    return {fmar(a.re, b.re, fmar(a.im, b.im, acc.re)), fmar(a.re, b.im, fmar(-a.im, b.re, acc.im))};
}
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R> __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b)
{
    return {fmar(a.re, b.re, a.im * b.im), fmar(a.re, b.im, -(a.im * b.re))};
}
// multiply by +i / -i
template <typename R> __device__ __forceinline__ cx<R> ti(cx<R> a) { return {-a.im, a.re}; }
template <typename R> __device__ __forceinline__ cx<R> tmi(cx<R> a) { return {a.im, -a.re}; }
template <typename R> __device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// Products whose operands come from binary16 storage.  a * b is written as
// fma(a, b, +0): the same value (up to the sign of an exact zero), but the
// compiler then folds the binary16 -> FP32 conversion of each operand into
// one mixed-precision multiply-add (v_fma_mix_f32) instead of converting
// first, which takes a conversion off every binary16 value used.
__device__ __forceinline__ float mul16(float a, float b) { return __builtin_fmaf(a, b, 0.0f); }

// --------------------------------------------------------------- planes --

constexpr int SB = 64;  // sites per block
__host__ __device__ constexpr long padded_sites(long n) { return (n + SB - 1) / SB * SB; }

template <typename T, int N> struct Planes {
    static constexpr int BYTES = N * (int)sizeof(T);
    static constexpr int K16 = BYTES / 16;
    static constexpr int TAIL = BYTES % 16;
    static constexpr int PER16 = 16 / (int)sizeof(T);
    static_assert(TAIL == 0 || TAIL == 8 || TAIL == 4, "unsupported tail");
    // bytes of the whole field over n sites
    __host__ __device__ static constexpr long field_bytes(long n) { return (long)BYTES * padded_sites(n); }
};

// REC, the site record's bytes, is the block stride; it differs from
// N*sizeof(T) only when a caller reads part of a record (the two 36-real
// halves of a clover block).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// NTL / NTS: non-temporal access (streamed data with no reuse, kept from
// displacing reused data in the caches).
template <typename V, bool NT> __device__ __forceinline__ V ld(const void *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    else return *reinterpret_cast<const V *>(p);
}
template <typename V, bool NT> __device__ __forceinline__ void st(void *p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    else *reinterpret_cast<V *>(p) = v;
}

template <typename T, int N, bool NTL = false, int REC = N * (int)sizeof(T)>
__device__ __forceinline__ void load_planes(const char *__restrict__ base, long s, long n, T *__restrict__ out)
{
    using PL = Planes<T, N>;
    const char *blk = base + (size_t)(s >> 6) * (size_t)(REC * SB);
    const uint32_t lane = (uint32_t)(s & 63);
#pragma unroll
    for (int k = 0; k < PL::K16; ++k) {
        const u32x4 q = ld<u32x4, NTL>(blk + k * 16 * SB + lane * 16u);
        __builtin_memcpy(out + k * PL::PER16, &q, 16);
    }
    const char *tl = blk + PL::K16 * 16 * SB;
    if constexpr (PL::TAIL == 8) {
        const u32x2 q = ld<u32x2, NTL>(tl + lane * 8u);
        __builtin_memcpy(out + PL::K16 * PL::PER16, &q, 8);
    } else if constexpr (PL::TAIL == 4) {
        const uint32_t q = ld<uint32_t, NTL>(tl + lane * 4u);
        __builtin_memcpy(out + PL::K16 * PL::PER16, &q, 4);
    }
}

template <typename T, int N, bool NTS = false, int REC = N * (int)sizeof(T)>
__device__ __forceinline__ void store_planes(char *__restrict__ base, long s, long n, const T *__restrict__ in)
{
    using PL = Planes<T, N>;
    char *blk = base + (size_t)(s >> 6) * (size_t)(REC * SB);
    const uint32_t lane = (uint32_t)(s & 63);
#pragma unroll
    for (int k = 0; k < PL::K16; ++k) {
        u32x4 q;
        __builtin_memcpy(&q, in + k * PL::PER16, 16);
        st<u32x4, NTS>(blk + k * 16 * SB + lane * 16u, q);
    }
    char *tl = blk + PL::K16 * 16 * SB;
    if constexpr (PL::TAIL == 8) {
        u32x2 q;
        __builtin_memcpy(&q, in + PL::K16 * PL::PER16, 8);
        st<u32x2, NTS>(tl + lane * 8u, q);
    } else if constexpr (PL::TAIL == 4) {
        uint32_t q;
        __builtin_memcpy(&q, in + PL::K16 * PL::PER16, 4);
        st<uint32_t, NTS>(tl + lane * 4u, q);
    }
}

// A spinor (12 complex = 24 reals) in compute precision R.
template <typename R> struct Spinor {
    cx<R> c[12];  // index spin*3 + colour
};

// Bytes of a packed spinor field over n sites, padded to whole blocks
// (FP16: the 48-byte records, then the scale plane).
__host__ __device__ constexpr long spinor_field_bytes(int p, long n)
{
    return (p == F64 ? 192 : p == F32 ? 96 : 52) * padded_sites(n);
}

template <int P>
__device__ __forceinline__ Spinor<typename PT<P>::R> load_spinor(const char *__restrict__ base, long s, long n)
{
    using S = typename PT<P>::S;
    using R = typename PT<P>::R;
    S raw[24];
    load_planes<S, 24>(base, s, n, raw);
    Spinor<R> o;
    if constexpr (PT<P>::scaled) {
        const float sc = *reinterpret_cast<const float *>(base + 48 * (size_t)padded_sites(n) + (uint32_t)s * 4u);
#pragma unroll
        for (int i = 0; i < 12; ++i) o.c[i] = cx<R>{mul16((R)raw[2 * i], sc), mul16((R)raw[2 * i + 1], sc)};
    } else {
#pragma unroll
        for (int i = 0; i < 12; ++i) o.c[i] = cx<R>{(R)raw[2 * i], (R)raw[2 * i + 1]};
    }
    return o;
}

// binary16 rounding of an FP32 value as a step of its own.  The empty
// register constraint keeps the compiler from folding the product that
// feeds the conversion into one mixed-precision multiply-add that rounds to
// binary16 once: it does so in some instantiations and not in others, and
// the results would then differ in the last bit between launch shapes.
__device__ __forceinline__ _Float16 to_f16(float x)
{
    asm("" : "+v"(x));
    return (_Float16)x;
}

template <int P, bool NTS = false>
__device__ __forceinline__ void store_spinor(char *__restrict__ base, long s, long n,
                                             const Spinor<typename PT<P>::R> &v)
{
    using S = typename PT<P>::S;
    using R = typename PT<P>::R;
    S raw[24];
    if constexpr (PT<P>::scaled) {
        R m = 0;
#pragma unroll
        for (int i = 0; i < 12; ++i) m = fmaxf(m, fmaxf(fabsf(v.c[i].re), fabsf(v.c[i].im)));
        const R inv = m > 0 ? (R)1 / m : (R)0;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            raw[2 * i] = to_f16(v.c[i].re * inv);
            raw[2 * i + 1] = to_f16(v.c[i].im * inv);
        }
        st<float, NTS>(base + 48 * (size_t)padded_sites(n) + (uint32_t)s * 4u, m);
    } else {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            raw[2 * i] = (S)v.c[i].re;
            raw[2 * i + 1] = (S)v.c[i].im;
        }
    }
    store_planes<S, 24, NTS>(base, s, n, raw);
}

// The values load_spinor returns after store_spinor(v): v itself for FP64
// and FP32 storage, v rounded to the scaled binary16 format otherwise
// (the same operations as the store and the load).
template <int P>
__device__ __forceinline__ Spinor<typename PT<P>::R> as_stored(const Spinor<typename PT<P>::R> &v)
{
    if constexpr (!PT<P>::scaled) {
        return v;
    } else {
        using S = typename PT<P>::S;
        using R = typename PT<P>::R;
        R m = 0;
#pragma unroll
        for (int i = 0; i < 12; ++i) m = fmaxf(m, fmaxf(fabsf(v.c[i].re), fabsf(v.c[i].im)));
        const R inv = m > 0 ? (R)1 / m : (R)0;
        const float sc = m;
        Spinor<R> o;
#pragma unroll
        for (int i = 0; i < 12; ++i)
            o.c[i] = cx<R>{mul16((R)to_f16(v.c[i].re * inv), sc), mul16((R)to_f16(v.c[i].im * inv), sc)};
        return o;
    }
}

// ------------------------------------------------------------- geometry --

// Lattice geometry of one checkerboarded lattice, passed by value.
struct Geom {
    int L[4];     // Lx, Ly, Lz, Lt
    int lxh;      // Lx / 2
    int vh;       // sites per parity
    double bc_re[4], bc_im[4];  // boundary phase per direction
};

// Coordinates of checkerboard site cb of parity p.
__device__ __forceinline__ void cb_coords(const Geom &g, int p, int cb, int c[4])
{
    int j = cb % g.lxh;
    int r = cb / g.lxh;
    c[1] = r % g.L[1];
    r /= g.L[1];
    c[2] = r % g.L[2];
    c[3] = r / g.L[2];
    c[0] = 2 * j + ((c[1] + c[2] + c[3] + p) & 1);
}

// Checkerboard index of the site with coordinates c.
__device__ __forceinline__ int cb_index(const Geom &g, const int c[4])
{
    return (c[0] >> 1) + g.lxh * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

}  // namespace lq

namespace lq {

// ------------------------------------------------------------ reductions --

// Sum over the 64 lanes of a wavefront (butterfly: same order every run).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a workgroup of NT threads; the result is valid in thread 0.
// Waves are combined through LDS in a fixed order, so the value does not
// depend on scheduling.  Every thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) r += lds[w];
    }
    __syncthreads();
    return r;
}

}  // namespace lq
