// su3.h -- FP64 colour matrices on the packed 18-real FP64 links, for the
// clover term (built from the plaquette leaves) and its force.
#pragma once

#include "fields.h"

namespace lq {

struct M3 {
    cx<double> e[9];
};

__device__ __forceinline__ M3 link_at(const Geom &g, const char *links64, const int c[4], int mu)
{
    const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
    M3 m;
    double raw[18];
    load_planes<double, 18>(links64 + (long)(p * 4 + mu) * link_bytes(F64, 18, g.vh), cb_index(g, c), g.vh, raw);
#pragma unroll
    for (int i = 0; i < 9; ++i) m.e[i] = cx<double>{raw[2 * i], raw[2 * i + 1]};
    return m;
}

__device__ __forceinline__ M3 mul(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            c.e[i * 3 + j] = a.e[i * 3 + 0] * b.e[0 * 3 + j] + a.e[i * 3 + 1] * b.e[1 * 3 + j] +
                             a.e[i * 3 + 2] * b.e[2 * 3 + j];
    return c;
}

__device__ __forceinline__ M3 dag(const M3 &a)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.e[i * 3 + j] = conj(a.e[j * 3 + i]);
    return c;
}

__device__ __forceinline__ M3 add(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 9; ++i) c.e[i] = a.e[i] + b.e[i];
    return c;
}

__device__ __forceinline__ void shift(const Geom &g, const int c[4], int mu, int dm, int nu, int dn, int o[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = c[k];
    o[mu] = (o[mu] + dm + g.L[mu]) % g.L[mu];
    o[nu] = (o[nu] + dn + g.L[nu]) % g.L[nu];
}

}  // namespace lq
