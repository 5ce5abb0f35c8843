// pack.hip -- conversions between the canonical FP64 layout of the ABI and
// the packed per-parity layouts of the kernels, and the bandwidth-reference
// copy kernel.  Links are compressed to 12 reals (two rows) when recon = 12,
// as in the caption of Table 2.
#include "wl_kernels.h"

namespace wl {

__device__ __forceinline__ size_t lex_site(const SysDesc &d, const Site &s)
{
    return (size_t)s.x + (size_t)d.L[0] * (s.y + (size_t)d.L[1] * (s.z + (size_t)d.L[2] * s.t));
}

template <int P>
__global__ __launch_bounds__(256) void k_pack_spinor(PackArgs a)
{
    using T = typename SpinorFmt<P>::real;
    const int lb = xcd_remap(blockIdx.x, a.nblocks);
    const BlkMap bm = a.map[lb];
    const VecDesc vd = a.vec[bm.v];
    const SysDesc sd = a.sys[vd.sys];
    const int cb = bm.lblk * (int)blockDim.x + (int)threadIdx.x;
    if (cb >= sd.Vh) return;
    const Site st = cb_coords(sd, cb, a.parity);
    const size_t V = 2 * (size_t)sd.Vh;
    const double *src = a.canon[vd.sys] + ((size_t)vd.rhs * V + lex_site(sd, st)) * 24;
    T v[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = (T)src[k];
    store_spinor<P>((typename SpinorFmt<P>::chunk *)a.f + (size_t)vd.site_off * SpinorFmt<P>::nchunk,
                    a.fn ? a.fn + vd.site_off : nullptr, sd.stride, cb, v);
}

template <int P>
__global__ __launch_bounds__(256) void k_unpack_spinor(PackArgs a)
{
    using T = typename SpinorFmt<P>::real;
    const int lb = xcd_remap(blockIdx.x, a.nblocks);
    const BlkMap bm = a.map[lb];
    const VecDesc vd = a.vec[bm.v];
    const SysDesc sd = a.sys[vd.sys];
    const int cb = bm.lblk * (int)blockDim.x + (int)threadIdx.x;
    if (cb >= sd.Vh) return;
    const Site st = cb_coords(sd, cb, a.parity);
    const size_t V = 2 * (size_t)sd.Vh;
    double *dst = (double *)a.canon[vd.sys] + ((size_t)vd.rhs * V + lex_site(sd, st)) * 24;
    T v[24];
    load_spinor<P>((const typename SpinorFmt<P>::chunk *)a.f + (size_t)vd.site_off * SpinorFmt<P>::nchunk,
                   a.fn ? a.fn + vd.site_off : nullptr, sd.stride, cb, v);
#pragma unroll
    for (int k = 0; k < 24; ++k) dst[k] = (double)v[k];
}

__global__ __launch_bounds__(256) void k_zero_canon(PackArgs a)
{
    const int lb = xcd_remap(blockIdx.x, a.nblocks);
    const BlkMap bm = a.map[lb];
    const VecDesc vd = a.vec[bm.v];
    const SysDesc sd = a.sys[vd.sys];
    const int cb = bm.lblk * (int)blockDim.x + (int)threadIdx.x;
    if (cb >= sd.Vh) return;
    const Site st = cb_coords(sd, cb, a.parity);
    const size_t V = 2 * (size_t)sd.Vh;
    double *dst = (double *)a.canon[vd.sys] + ((size_t)vd.rhs * V + lex_site(sd, st)) * 24;
#pragma unroll
    for (int k = 0; k < 24; ++k) dst[k] = 0.0;
}

template <int P, int R>
__global__ __launch_bounds__(256) void k_pack_gauge(const double *U, void *out, SysDesc d)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 2 * d.Vh) return;
    const int parity = tid / d.Vh, cb = tid - parity * d.Vh;
    const Site st = cb_coords(d, cb, parity);
    const size_t s = lex_site(d, st);
    constexpr int NCH = LinkFmt<P, R>::nchunk;
    using CH = typename LinkFmt<P, R>::chunk;
    for (int mu = 0; mu < 4; ++mu) {
        double u[18];
        const double *src = U + (s * 4 + mu) * 18;
        for (int k = 0; k < 18; ++k) u[k] = src[k];
        store_link<P, R>((CH *)out + (size_t)((parity * 4 + mu) * NCH) * d.gstride, d.gstride, cb, u);
    }
}

// Reference copy for the achievable-bandwidth figure: one 16-byte element per
// thread with non-temporal loads and stores (the fastest plain copy measured
// on gfx950: one element per thread beats grid-stride loops and unrolling)
__global__ __launch_bounds__(256) void k_copy_bw(const float4 *__restrict__ in, float4 *__restrict__ out, size_t n)
{
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) WL_NT_STORE(nt_f4, WL_NT_LOAD(nt_f4, in + i), out + i);
}

// The same copy with ordinary (cached) loads and stores: operands small enough
// for the last-level cache stay there between launches.
__global__ __launch_bounds__(256) void k_copy_cached(const float4 *__restrict__ in, float4 *__restrict__ out, size_t n)
{
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

// Read-only reference: each thread sums four 16-byte elements a grid apart
// with ordinary loads; the sum is stored only when it equals a value a zeroed
// buffer never produces, so no store reaches memory.
__global__ __launch_bounds__(256) void k_read_cached(const float4 *__restrict__ in, float *__restrict__ out, size_t n)
{
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x, st = (size_t)gridDim.x * blockDim.x;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i + k * st < n) {
            const float4 v = in[i + k * st];
            s += (v.x + v.y) + (v.z + v.w);
        }
    if (s == 1.0f) out[blockIdx.x] = s;
}

template <int P>
static hipError_t launch_pack_t(bool unpack, const PackArgs &a, int block, hipStream_t s)
{
    if (unpack)
        hipLaunchKernelGGL(k_unpack_spinor<P>, dim3(a.nblocks), dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL(k_pack_spinor<P>, dim3(a.nblocks), dim3(block), 0, s, a);
    return hipGetLastError();
}

static hipError_t launch_pack_any(bool unpack, int prec, const PackArgs &a, int block, hipStream_t s)
{
    switch (prec) {
    case P_F64: return launch_pack_t<P_F64>(unpack, a, block, s);
    case P_F32: return launch_pack_t<P_F32>(unpack, a, block, s);
    case P_F16: return launch_pack_t<P_F16>(unpack, a, block, s);
    case P_BF16: return launch_pack_t<P_BF16>(unpack, a, block, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pack_spinor(int prec, const PackArgs &a, int block, hipStream_t s)
{
    return launch_pack_any(false, prec, a, block, s);
}

hipError_t launch_unpack_spinor(int prec, const PackArgs &a, int block, hipStream_t s)
{
    return launch_pack_any(true, prec, a, block, s);
}

hipError_t launch_zero_canon(const PackArgs &a, int block, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_canon, dim3(a.nblocks), dim3(block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_gauge(int prec, int recon, const double *U, void *out, const SysDesc &d, hipStream_t s)
{
    const int n = 2 * d.Vh, blk = 256, grid = (n + blk - 1) / blk;
    if (prec == P_F64 && recon == 18) hipLaunchKernelGGL((k_pack_gauge<P_F64, 18>), dim3(grid), dim3(blk), 0, s, U, out, d);
    else if (prec == P_F64 && recon == 12) hipLaunchKernelGGL((k_pack_gauge<P_F64, 12>), dim3(grid), dim3(blk), 0, s, U, out, d);
    else if (prec == P_F32 && recon == 18) hipLaunchKernelGGL((k_pack_gauge<P_F32, 18>), dim3(grid), dim3(blk), 0, s, U, out, d);
    else if (prec == P_F32 && recon == 12) hipLaunchKernelGGL((k_pack_gauge<P_F32, 12>), dim3(grid), dim3(blk), 0, s, U, out, d);
    else if (prec == P_F16 && recon == 12) hipLaunchKernelGGL((k_pack_gauge<P_F16, 12>), dim3(grid), dim3(blk), 0, s, U, out, d);
    else if (prec == P_BF16 && recon == 12) hipLaunchKernelGGL((k_pack_gauge<P_BF16, 12>), dim3(grid), dim3(blk), 0, s, U, out, d);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_copy_bw(int mode, const void *in, void *out, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / sizeof(float4);
    const int blk = 256;
    // the read-only kernel takes four elements per thread and stores at most
    // one float per block into `out` (which holds `bytes` bytes)
    const size_t grid = mode == 2 ? (n / 4 + blk - 1) / blk : (n + blk - 1) / blk;
    if (grid > 0x7FFFFFFFu || grid == 0) return hipErrorInvalidValue;
    if (mode == 0)
        hipLaunchKernelGGL(k_copy_bw, dim3((unsigned)grid), dim3(blk), 0, s, (const float4 *)in, (float4 *)out, n);
    else if (mode == 1)
        hipLaunchKernelGGL(k_copy_cached, dim3((unsigned)grid), dim3(blk), 0, s, (const float4 *)in, (float4 *)out, n);
    else if (mode == 2)
        hipLaunchKernelGGL(k_read_cached, dim3((unsigned)grid), dim3(blk), 0, s, (const float4 *)in, (float *)out, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace wl
