// wl_reduce.h -- deterministic FP64 reductions for wave64 blocks.
//
// Per block: 64-lane butterfly shuffles, then one LDS slot per wave, then the
// first wave; the block's partial goes to a per-(vector, block) slot, and a
// finishing kernel adds each vector's partials in a fixed order, so the result
// does not depend on block scheduling.
#pragma once

#include "wl_launch.h"

namespace wl {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.  blockDim.x must be a
// multiple of 64 and at most 1024.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double lds[16];
    __syncthreads();  // lds may still be read by a previous call
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (w == 0) {
        r = l < (int)(blockDim.x >> 6) ? lds[l] : 0.0;
        r = wave_sum(r);
    }
    return r;
}

__device__ __forceinline__ void red_finalize(const RedSpec &r, int v, double s)
{
    if (!isfinite(s) && r.bad) r.bad[v] |= 1;
    switch (r.kind) {
    case RED_STORE:
        r.dst[v] = s;
        break;
    case RED_ALPHA:
        r.alpha[v] = s > 0.0 ? r.gam[v] / s : 0.0;
        break;
    case RED_BETA: {
        const double g = r.gam[v];
        r.beta[v] = g > 0.0 ? s / g : 0.0;
        r.gam[v] = s;
        break;
    }
    case RED_GAMMA:
        r.gam[v] = s;
        break;
    case RED_ACCUM:
        r.dst[v] += s;
        break;
    default:
        break;
    }
}

// Called by every thread of the block (uniform control flow) with its own
// contribution `mine`: the block's sum goes to its partial slot.  The slots of
// a vector are added in a fixed order by k_red_finalize after the producing
// kernel ends; the kernel boundary makes the partials visible without any
// device-scope fence inside the producer (on gfx950 such a fence writes back
// the XCD's L2 and costs far more than a separate finishing launch).
__device__ __forceinline__ void block_reduce_store(const RedSpec &r, int pslot0, int lblk, double mine)
{
    const double bs = block_sum(mine);
    if (threadIdx.x == 0) r.partials[pslot0 + lblk] = bs;
}

template <class T> __device__ __forceinline__ double site_norm2(const T o[24])
{
    T s = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) s += o[k] * o[k];
    return (double)s;
}

}  // namespace wl
