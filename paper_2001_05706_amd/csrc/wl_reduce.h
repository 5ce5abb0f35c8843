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

// Sums over the block of nv <= 3 values per thread, valid in thread 0: one
// pass of LDS traffic for all of them.
__device__ __forceinline__ void block_sum_n(double *v, int nv)
{
    __shared__ double lds[3][16];
    __syncthreads();  // lds may still be read by a previous call
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int k = 0; k < nv; ++k) {
        v[k] = wave_sum(v[k]);
        if (l == 0) lds[k][w] = v[k];
    }
    __syncthreads();
    if (w == 0)
        for (int k = 0; k < nv; ++k) v[k] = wave_sum(l < (int)(blockDim.x >> 6) ? lds[k][l] : 0.0);
}

// The values the finishing step of a reduction reads besides the sums
// (loaded before the sums are complete, so that their latency overlaps).
struct RedIn {
    double a = 0.0, b = 0.0;
};

__device__ __forceinline__ RedIn red_prefetch(const RedSpec &r, int v)
{
    RedIn in;
    const double *sc = r.sc;
    const int n = r.nvec;
    switch (r.kind) {
    case RED_ALPHA:
    case RED_BETA: in.a = sc[SC_GAM * n + v]; break;
    case RED_ACCUM: in.a = r.dst[v]; break;
    case RED_BICG_ALPHA:
        in.a = sc[SC_RHO_RE * n + v];
        in.b = sc[SC_RHO_IM * n + v];
        break;
    case RED_CACCUM:
        in.a = r.dst[2 * v];
        in.b = r.dst[2 * v + 1];
        break;
    default: break;
    }
    return in;
}

__device__ __forceinline__ void red_finalize(const RedSpec &r, int v, const double *s, const RedIn &in)
{
    bool finite = true;
    for (int k = 0; k < r.nv; ++k) finite = finite && isfinite(s[k]);
    double *sc = r.sc;
    const int n = r.nvec;
#define WL_SC(slot) sc[(slot) * n + v]
    switch (r.kind) {
    case RED_STORE: r.dst[v] = s[0]; break;
    case RED_ALPHA: WL_SC(SC_ALPHA) = s[0] > 0.0 ? in.a / s[0] : 0.0; break;
    case RED_BETA: {
        const double g = in.a;
        WL_SC(SC_BETA) = g > 0.0 ? s[0] / g : 0.0;
        WL_SC(SC_GAM) = s[0];
        break;
    }
    case RED_GAMMA: WL_SC(SC_GAM) = s[0]; break;
    case RED_ACCUM: r.dst[v] = in.a + s[0]; break;
    case RED_CDOT_RHO:
        WL_SC(SC_RHO_RE) = s[0];
        WL_SC(SC_RHO_IM) = s[1];
        break;
    case RED_BICG_ALPHA: {
        // alpha = rho / d, a zero d is a breakdown: reported as non-finite
        const double dr = s[0], di = s[1], d2 = dr * dr + di * di;
        const double rr = in.a, ri = in.b;
        if (!(d2 > 0.0)) finite = false;
        WL_SC(SC_AL_RE) = d2 > 0.0 ? (rr * dr + ri * di) / d2 : 0.0;
        WL_SC(SC_AL_IM) = d2 > 0.0 ? (ri * dr - rr * di) / d2 : 0.0;
        WL_SC(SC_RHOP_RE) = rr;
        WL_SC(SC_RHOP_IM) = ri;
        break;
    }
    case RED_BICG_OMEGA:
        if (!(s[2] > 0.0)) finite = false;
        WL_SC(SC_OM_RE) = s[2] > 0.0 ? s[0] / s[2] : 0.0;
        WL_SC(SC_OM_IM) = s[2] > 0.0 ? s[1] / s[2] : 0.0;
        break;
    case RED_BICG_INIT:
        WL_SC(SC_RHO_RE) = WL_SC(SC_RHOP_RE) = s[0];
        WL_SC(SC_RHO_IM) = WL_SC(SC_RHOP_IM) = s[1];
        WL_SC(SC_AL_RE) = WL_SC(SC_OM_RE) = 1.0;
        WL_SC(SC_AL_IM) = WL_SC(SC_OM_IM) = 0.0;
        if (!(s[0] * s[0] + s[1] * s[1] > 0.0)) finite = false;
        break;
    case RED_BICG_RHO:
        WL_SC(SC_RHO_RE) = s[0];
        WL_SC(SC_RHO_IM) = s[1];
        r.dst[v] = s[2];
        break;
    case RED_CSTORE:
        r.dst[2 * v] = s[0];
        r.dst[2 * v + 1] = s[1];
        break;
    case RED_CACCUM:
        r.dst[2 * v] = in.a + s[0];
        r.dst[2 * v + 1] = in.b + s[1];
        break;
    default: break;
    }
#undef WL_SC
    if (!finite && r.bad) r.bad[v] |= 1;
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
    if (threadIdx.x == 0) r.partials[(size_t)(pslot0 + lblk) * r.nv] = bs;
}

// nv values per thread (nv = r.nv <= 3)
__device__ __forceinline__ void block_reduce_store_n(const RedSpec &r, int pslot0, int lblk, const double *mine)
{
    for (int k = 0; k < r.nv; ++k) {
        const double bs = block_sum(mine[k]);
        if (threadIdx.x == 0) r.partials[(size_t)(pslot0 + lblk) * r.nv + k] = bs;
    }
}

// Per-wave variant (blocks whose waves serve different vectors): the wave's
// sum goes to its own vector's partial slot; every lane of the wave calls it.
__device__ __forceinline__ void wave_reduce_store_n(const RedSpec &r, int pslot0, int lblk, const double *mine)
{
    for (int k = 0; k < r.nv; ++k) {
        const double ws = wave_sum(mine[k]);
        if ((threadIdx.x & 63) == 0) r.partials[(size_t)(pslot0 + lblk) * r.nv + k] = ws;
    }
}

// <a, b> = sum conj(a) b over one site (12 complex numbers)
template <class T> __device__ __forceinline__ void site_cdot(const T a[24], const T b[24], double &re, double &im)
{
    // explicit fused multiply-adds: every instantiation rounds alike (left to
    // the compiler, which of two products gets fused can differ between
    // instantiations of the same source)
    T sr = 0, si = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        sr = fmadd(a[2 * k], b[2 * k], sr);
        sr = fmadd(a[2 * k + 1], b[2 * k + 1], sr);
        si = fmadd(a[2 * k], b[2 * k + 1], si);
        si = fmadd(-a[2 * k + 1], b[2 * k], si);
    }
    re = (double)sr;
    im = (double)si;
}

template <class T> __device__ __forceinline__ double site_norm2(const T o[24])
{
    T s = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) s += o[k] * o[k];
    return (double)s;
}

}  // namespace wl
