// blas.hip -- fused BLAS-1 kernels of the solvers with per-vector scalars
// read from device memory and fused FP64 norm reductions (the vector
// operations GWU-code ran through Thrust, Section 3, and QUDA's multi-vector
// BLAS/reduction kernels, Section 2).
//
// Products are formed in the storage arithmetic (FP32 for FP32/FP16/BF16,
// FP64 for FP64); norms accumulate per site in that arithmetic and across
// sites in FP64 with the deterministic block reduction.
#include "wl_reduce.h"
#include "wl_kernels.h"

namespace wl {

// Takes the descriptor values as operands, so that their loads are all issued
// before this point (the compiler would otherwise sink each load to its first
// use behind the early exits, one memory round trip after another).
__device__ __forceinline__ void blas_issued(int a, int b, int c, int d, int e)
{
    asm volatile("" ::"s"(a), "s"(b), "s"(c), "s"(d), "s"(e));
}

// Streaming hint for the store of the field the next hop reads as its
// neighbour input (p or r in CGNR, p or s in BiCGStab): plain in FP32 and FP64,
// so that the field waits for the hop in the last-level cache (32^3x64 FP32
// CGNR 3% faster); with half-precision fields the plain store
// slowed the hops as much as it sped up the updates, and the hops' share of
// the traffic is what the links' place in that cache is kept for.
template <int P, bool NT> constexpr bool kNextHopNT = NT && (P == P_F16 || P == P_BF16);

// The block's vector vi, its descriptors and its logical block.  Every kernel
// has the template flag ONE: instantiated true for a set of one vector, whose
// descriptors sit at index 0, so that their loads and the block map's go out
// together (two dependent rounds fewer at the start of every wave).
#define WL_BLAS_PROLOGUE                                              \
    const int lb = xcd_remap(blockIdx.x, a.nblocks);                  \
    const BlkMap bm = a.map[lb];                                      \
    const int vi = ONE ? 0 : bm.v;                                    \
    const VecDesc vd = a.vec[vi];                                     \
    const SysDesc sd = a.sys[ONE ? 0 : vd.sys];                       \
    const int act = a.active ? a.active[vi] : 1;                      \
    if constexpr (ONE) blas_issued(bm.lblk, vd.site_off, sd.Vh, sd.stride, act); \
    if (!act) return;                                                 \
    const int cb = bm.lblk * (int)blockDim.x + (int)threadIdx.x;      \
    const bool live = cb < sd.Vh;

template <int P> __device__ __forceinline__ const void *vbase(const void *f, const VecDesc &vd)
{
    return (const typename SpinorFmt<P>::chunk *)f + (size_t)vd.site_off * SpinorFmt<P>::nchunk;
}
template <int P> __device__ __forceinline__ void *vbase(void *f, const VecDesc &vd)
{
    return (typename SpinorFmt<P>::chunk *)f + (size_t)vd.site_off * SpinorFmt<P>::nchunk;
}
__device__ __forceinline__ float *nbase(float *n, const VecDesc &vd) { return n ? n + vd.site_off : nullptr; }

// field j of the launch for vector vd: a shared single vector when its bcast bit is set
template <int P> __device__ __forceinline__ const void *fbase(const BlasArgs &a, int j, const VecDesc &vd)
{
    return (a.bcast >> j) & 1 ? a.f[j] : vbase<P>(a.f[j], vd);
}

template <int P, bool ONE = false, bool NT = false>
__global__ __launch_bounds__(256) void k_cg_update(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    double nrm = 0.0;
    if (live) {
        const T al = (T)a.s0[vi];
        T x[24], p[24], r[24], q[24];
        load_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
        load_spinor<P, NT>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, p);
        load_spinor<P, NT>(vbase<P>(a.f[2], vd), nbase(a.fn[2], vd), sd.stride, cb, r);
        load_spinor<P, NT>(vbase<P>(a.f[3], vd), nbase(a.fn[3], vd), sd.stride, cb, q);
#pragma unroll
        for (int k = 0; k < 24; ++k) {
            x[k] += al * p[k];
            r[k] -= al * q[k];
        }
        store_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
        store_spinor<P, NT>(vbase<P>(a.f[2], vd), nbase(a.fn[2], vd), sd.stride, cb, r);
        nrm = site_norm2(r);
    }
    if (a.red.kind != RED_NONE) block_reduce_store(a.red, vd.pslot0, bm.lblk, nrm);
}

template <int P, bool ONE = false, bool NT = false>
__global__ __launch_bounds__(256) void k_xpay(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    const T be = (T)a.s0[vi];
    T p[24], s[24];
    load_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, p);
    load_spinor<P, NT>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, s);
#pragma unroll
    for (int k = 0; k < 24; ++k) p[k] = s[k] + be * p[k];
    store_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, p);
}

// CGNR with the solution update folded into the direction update: the
// residual step alone here, x += alpha p with p = s + beta p below
template <int P, bool ONE = false, bool NT = false>
__global__ __launch_bounds__(256) void k_r_update(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    double nrm = 0.0;
    if (live) {
        const T al = (T)a.s0[vi];
        T r[24], q[24];
        load_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, r);
        load_spinor<P, NT>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, q);
#pragma unroll
        for (int k = 0; k < 24; ++k) r[k] -= al * q[k];
        // r is the neighbour input of the next hop (of M^+)
        store_spinor<P, kNextHopNT<P, NT>>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, r);
        nrm = site_norm2(r);
    }
    if (a.red.kind != RED_NONE) block_reduce_store(a.red, vd.pslot0, bm.lblk, nrm);
}

template <int P, bool ONE = false, bool NT = false>
__global__ __launch_bounds__(256) void k_xpay_x(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    const T be = (T)a.s0[vi];
    const T al = (T)a.sc[SC_ALPHA * a.nvec + vi];
    T p[24], s[24], x[24];
    load_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, p);
    load_spinor<P, NT>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, s);
    load_spinor<P, NT>(vbase<P>(a.f[2], vd), nbase(a.fn[2], vd), sd.stride, cb, x);
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        x[k] += al * p[k];
        p[k] = s[k] + be * p[k];
    }
    store_spinor<P, NT>(vbase<P>(a.f[2], vd), nbase(a.fn[2], vd), sd.stride, cb, x);
    // p is the neighbour input of the next hop (of M)
    store_spinor<P, kNextHopNT<P, NT>>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, p);
}

template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_accum(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    double y[24];
    T x[24];
    load_spinor<P_F64>(vbase<P_F64>(a.f[0], vd), nullptr, sd.stride, cb, y);
    load_spinor<P>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, x);
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        y[k] += (double)x[k];
        x[k] = 0;
    }
    store_spinor<P_F64>(vbase<P_F64>(a.f[0], vd), nullptr, sd.stride, cb, y);
    store_spinor<P>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, x);
}

template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_norm2(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    double nrm = 0.0;
    if (live) {
        T x[24];
        load_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
        nrm = site_norm2(x);
    }
    block_reduce_store(a.red, vd.pslot0, bm.lblk, nrm);
}

template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_zero(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    T x[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) x[k] = 0;
    store_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
}

template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_fill(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    T x[24];
    uint32_t h = (uint32_t)(vd.site_off + cb) * 2654435761u + 12345u;
#pragma unroll
    for (int k = 0; k < 24; ++k) {
        h ^= h << 13;
        h ^= h >> 17;
        h ^= h << 5;
        x[k] = (T)((float)(h & 0xFFFFu) * (1.0f / 32768.0f) - 1.0f);
    }
    store_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
}

template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_scale_rsqrt(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    const double n2 = a.s0[vi];
    const T f = (T)(n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0);
    T x[24];
    load_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
#pragma unroll
    for (int k = 0; k < 24; ++k) x[k] *= f;
    store_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
}

// complex scalar of vector v from two slots
__device__ __forceinline__ void cscal(const BlasArgs &a, int re_slot, int v, double &re, double &im)
{
    re = a.sc[(size_t)re_slot * a.nvec + v];
    im = a.sc[(size_t)(re_slot + 1) * a.nvec + v];
}

// y = z * x for complex z and a site of 12 complex numbers.  The fused
// multiply-adds are written out, so that the streamed and plain
// instantiations of a kernel round alike.
template <class T> __device__ __forceinline__ void cmul_site(T zr, T zi, const T x[24], T y[24])
{
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        y[2 * k] = fmadd(zr, x[2 * k], -(zi * x[2 * k + 1]));
        y[2 * k + 1] = fmadd(zr, x[2 * k + 1], zi * x[2 * k]);
    }
}

template <int P, bool ONE = false, bool NT = false>
__global__ __launch_bounds__(256) void k_bicg_p(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    double rr, ri, pr, pi, ar, ai, orr, oi;
    cscal(a, SC_RHO_RE, vi, rr, ri);
    cscal(a, SC_RHOP_RE, vi, pr, pi);
    cscal(a, SC_AL_RE, vi, ar, ai);
    cscal(a, SC_OM_RE, vi, orr, oi);
    // beta = (rho / rho_prev) (alpha / omega), fused multiply-adds written out
    const double d1 = fma(pr, pr, pi * pi), d2 = fma(orr, orr, oi * oi);
    const double q1r = fma(rr, pr, ri * pi) / d1, q1i = fma(ri, pr, -(rr * pi)) / d1;
    const double q2r = fma(ar, orr, ai * oi) / d2, q2i = fma(ai, orr, -(ar * oi)) / d2;
    const T br = (T)fma(q1r, q2r, -(q1i * q2i)), bi = (T)fma(q1r, q2i, q1i * q2r);
    T p[24], r[24], v[24], t[24];
    load_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, p);
    load_spinor<P, NT>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, r);
    load_spinor<P, NT>(vbase<P>(a.f[2], vd), nbase(a.fn[2], vd), sd.stride, cb, v);
    cmul_site((T)orr, (T)oi, v, t);  // omega v
#pragma unroll
    for (int k = 0; k < 24; ++k) t[k] = p[k] - t[k];
    cmul_site(br, bi, t, p);  // beta (p - omega v)
#pragma unroll
    for (int k = 0; k < 24; ++k) p[k] += r[k];
    // p is the neighbour input of the next hop
    store_spinor<P, kNextHopNT<P, NT>>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, p);
}

template <int P, bool ONE = false, bool NT = false>
__global__ __launch_bounds__(256) void k_bicg_s(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    double ar, ai;
    cscal(a, SC_AL_RE, vi, ar, ai);
    T r[24], v[24], av[24];
    load_spinor<P, NT>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, r);
    load_spinor<P, NT>(vbase<P>(a.f[2], vd), nbase(a.fn[2], vd), sd.stride, cb, v);
    cmul_site((T)ar, (T)ai, v, av);
#pragma unroll
    for (int k = 0; k < 24; ++k) r[k] -= av[k];
    // s is the neighbour input of the next hop
    store_spinor<P, kNextHopNT<P, NT>>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, r);
}

template <int P, bool ONE = false, bool NT = false>
__global__ __launch_bounds__(256) void k_bicg_xr(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    double rv[3] = {0.0, 0.0, 0.0};
    if (live) {
        double ar, ai, orr, oi;
        cscal(a, SC_AL_RE, vi, ar, ai);
        cscal(a, SC_OM_RE, vi, orr, oi);
        T x[24], y[24], z[24], w[24];
        load_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
        load_spinor<P, NT>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, y);  // p
        cmul_site((T)ar, (T)ai, y, z);
#pragma unroll
        for (int k = 0; k < 24; ++k) x[k] += z[k];
        load_spinor<P, NT>(vbase<P>(a.f[2], vd), nbase(a.fn[2], vd), sd.stride, cb, y);  // s
        cmul_site((T)orr, (T)oi, y, z);
#pragma unroll
        for (int k = 0; k < 24; ++k) x[k] += z[k];
        store_spinor<P, NT>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
        load_spinor<P, NT>(vbase<P>(a.f[4], vd), nbase(a.fn[4], vd), sd.stride, cb, w);  // t
        cmul_site((T)orr, (T)oi, w, z);
#pragma unroll
        for (int k = 0; k < 24; ++k) y[k] -= z[k];  // r = s - omega t
        store_spinor<P, NT>(vbase<P>(a.f[3], vd), nbase(a.fn[3], vd), sd.stride, cb, y);
        load_spinor<P, NT>(vbase<P>(a.f[5], vd), nbase(a.fn[5], vd), sd.stride, cb, w);  // rhat
        site_cdot(w, y, rv[0], rv[1]);
        rv[2] = site_norm2(y);
    }
    block_reduce_store_n(a.red, vd.pslot0, bm.lblk, rv);
}

template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_cdot(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    double rv[3] = {0.0, 0.0, 0.0};
    if (live) {
        T x[24], y[24];
        load_spinor<P>(fbase<P>(a, 0, vd), nbase(a.fn[0], vd), sd.stride, cb, x);
        load_spinor<P>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, y);
        site_cdot(x, y, rv[0], rv[1]);
    }
    block_reduce_store_n(a.red, vd.pslot0, bm.lblk, rv);
}

// y += z x (G5: y += z g5 x) with the complex z of this vector from s0
template <int P, bool G5, bool ONE = false>
__global__ __launch_bounds__(256) void k_caxpy(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    const T zr = (T)a.s0[2 * vi], zi = (T)a.s0[2 * vi + 1];
    T x[24], y[24];
    load_spinor<P>(fbase<P>(a, 1, vd), nbase(a.fn[1], vd), sd.stride, cb, x);
    load_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, y);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const T s = (G5 && k >= 6) ? (T)-1 : (T)1;
        y[2 * k] += s * (zr * x[2 * k] - zi * x[2 * k + 1]);
        y[2 * k + 1] += s * (zr * x[2 * k + 1] + zi * x[2 * k]);
    }
    store_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, y);
}

// y_v = sum_j T[j + nvec v] x_j over the vectors j of a single-system set
// (vector j starts j strides into the field); T complex in s0
template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_rot(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    using CH = typename SpinorFmt<P>::chunk;
    WL_BLAS_PROLOGUE
    if (!live) return;
    T y[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) y[k] = 0;
    for (int j = 0; j < a.nvec; ++j) {
        const double *t = a.s0 + 2 * ((size_t)j + (size_t)a.nvec * vi);
        const T tr = (T)t[0], ti = (T)t[1];
        T x[24];
        load_spinor<P>((const CH *)a.f[1] + (size_t)j * sd.stride * SpinorFmt<P>::nchunk,
                       a.fn[1] ? a.fn[1] + (size_t)j * sd.stride : nullptr, sd.stride, cb, x);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            y[2 * k] += tr * x[2 * k] - ti * x[2 * k + 1];
            y[2 * k + 1] += tr * x[2 * k + 1] + ti * x[2 * k];
        }
    }
    store_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, y);
}

// y = g5 x: spins 2 and 3 (the last 12 reals of a site) change sign
template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_g5copy(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    T x[24];
    load_spinor<P>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, x);
#pragma unroll
    for (int k = 12; k < 24; ++k) x[k] = -x[k];
    store_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
}

// y = A^{-1} x at the sites of parity a.parity (FP64 term for FP64 fields,
// FP32 otherwise); systems without a clover term copy
template <int P, bool ONE = false>
__global__ __launch_bounds__(256) void k_clov_inv(BlasArgs a)
{
    using T = typename SpinorFmt<P>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    constexpr int CP = clover_prec<P>();
    T x[24];
    load_spinor<P>(vbase<P>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, x);
    if (sd.clovinv) clover_apply<CP>(clover_parity<CP>(sd.clovinv, a.parity, sd.stride), sd.stride, cb, x);
    store_spinor<P>(vbase<P>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, x);
}

template <int PD, int PS, bool ONE = false>
__global__ __launch_bounds__(256) void k_convert(BlasArgs a)
{
    using TS = typename SpinorFmt<PS>::real;
    using TD = typename SpinorFmt<PD>::real;
    WL_BLAS_PROLOGUE
    if (!live) return;
    TS x[24];
    TD y[24];
    load_spinor<PS>(vbase<PS>(a.f[1], vd), nbase(a.fn[1], vd), sd.stride, cb, x);
#pragma unroll
    for (int k = 0; k < 24; ++k) y[k] = (TD)x[k];
    store_spinor<PD>(vbase<PD>(a.f[0], vd), nbase(a.fn[0], vd), sd.stride, cb, y);
}

// Solver-iteration kernels come in four instantiations: one-vector sets (see
// WL_BLAS_PROLOGUE) and streamed fields.  Their field accesses carry the
// non-temporal hint when the set's fields are large against the 256 MB
// last-level cache (ExecSet::stream_fields): each field is streamed once per
// launch, and without the hint it displaces the links, which the four hops of
// an iteration re-read from that cache.
#define WL_LAUNCH_ITER(K)                                                     \
    do {                                                                      \
        if (a.one && a.stream) hipLaunchKernelGGL((K<P, true, true>), g, b, 0, s, a); \
        else if (a.one) hipLaunchKernelGGL((K<P, true, false>), g, b, 0, s, a);      \
        else if (a.stream) hipLaunchKernelGGL((K<P, false, true>), g, b, 0, s, a);   \
        else hipLaunchKernelGGL((K<P, false, false>), g, b, 0, s, a);                \
    } while (0)

template <int P>
static hipError_t launch_blas_t(int op, const BlasArgs &a, int block, hipStream_t s)
{
    dim3 g(a.nblocks), b(block);
    switch (op) {
    case BL_CG_UPDATE: WL_LAUNCH_ITER(k_cg_update); break;
    case BL_XPAY: WL_LAUNCH_ITER(k_xpay); break;
    case BL_ACCUM: hipLaunchKernelGGL(k_accum<P>, g, b, 0, s, a); break;
    case BL_NORM2: hipLaunchKernelGGL(k_norm2<P>, g, b, 0, s, a); break;
    case BL_ZERO: hipLaunchKernelGGL(k_zero<P>, g, b, 0, s, a); break;
    case BL_COPY: hipLaunchKernelGGL((k_convert<P, P>), g, b, 0, s, a); break;
    case BL_FILL: hipLaunchKernelGGL(k_fill<P>, g, b, 0, s, a); break;
    case BL_SCALE_RSQRT: hipLaunchKernelGGL(k_scale_rsqrt<P>, g, b, 0, s, a); break;
    case BL_BICG_P: WL_LAUNCH_ITER(k_bicg_p); break;
    case BL_BICG_S: WL_LAUNCH_ITER(k_bicg_s); break;
    case BL_BICG_XR: WL_LAUNCH_ITER(k_bicg_xr); break;
    case BL_CDOT: hipLaunchKernelGGL(k_cdot<P>, g, b, 0, s, a); break;
    case BL_G5COPY: hipLaunchKernelGGL(k_g5copy<P>, g, b, 0, s, a); break;
    case BL_CLOV_INV: hipLaunchKernelGGL(k_clov_inv<P>, g, b, 0, s, a); break;
    case BL_CAXPY: hipLaunchKernelGGL((k_caxpy<P, false>), g, b, 0, s, a); break;
    case BL_CAXPY_G5: hipLaunchKernelGGL((k_caxpy<P, true>), g, b, 0, s, a); break;
    case BL_ROT: hipLaunchKernelGGL(k_rot<P>, g, b, 0, s, a); break;
    case BL_R_UPDATE: WL_LAUNCH_ITER(k_r_update); break;
    case BL_XPAY_X: WL_LAUNCH_ITER(k_xpay_x); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One block per vector: fixed-order sum of the vector's partials, then the
// finishing step (scalar update) of the reduction kind.
template <int NV>
__global__ __launch_bounds__(1024) void k_red_finalize(RedSpec r, const VecDesc *vec, const int32_t *active)
{
    const int v = blockIdx.x;
    if (active && !active[v]) return;
    RedIn in;
    if (threadIdx.x == 0) in = red_prefetch(r, v);
    const VecDesc vd = vec[v];
    const double *p = r.partials + (size_t)vd.pslot0 * NV;
    const int bd = (int)blockDim.x;
    double tot[3] = {0.0, 0.0, 0.0};
    // four partials per step, all loaded before any is added (their latencies
    // overlap), then the tail; the order of the additions is fixed
    int i = threadIdx.x;
    for (; i + 3 * bd < vd.nblk; i += 4 * bd) {
        double w[4][NV];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < NV; ++k) w[u][k] = p[(size_t)(i + u * bd) * NV + k];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < NV; ++k) tot[k] += w[u][k];
    }
    for (; i < vd.nblk; i += bd)
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] += p[(size_t)i * NV + k];
    block_sum_n(tot, NV);
    if (threadIdx.x == 0) red_finalize(r, v, tot, in);
}

// Deferred |r|^2 of k iterations: block (v, j) sums row j of the per-iteration
// partials of vector v in a fixed order into hist[j * nvec + v].
__global__ __launch_bounds__(256) void k_hist_finalize(const double *partials, size_t row, const VecDesc *vec,
                                                       const int32_t *active, int nvec, double *hist, int32_t *bad)
{
    const int v = blockIdx.x, j = blockIdx.y;
    if (active && !active[v]) return;
    const VecDesc vd = vec[v];
    const double *p = partials + (size_t)j * row + vd.pslot0;
    double s = 0.0;
    for (int i = threadIdx.x; i < vd.nblk; i += blockDim.x) s += p[i];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        hist[(size_t)j * nvec + v] = s;
        if (!isfinite(s) && bad) bad[v] |= 1;
    }
}

hipError_t launch_hist_finalize(const double *partials, size_t row, const VecDesc *vec, const int32_t *active, int nvec,
                                int k, double *hist, int32_t *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_hist_finalize, dim3(nvec, k), dim3(256), 0, s, partials, row, vec, active, nvec, hist, bad);
    return hipGetLastError();
}

hipError_t launch_red_finalize(const RedSpec &r, const VecDesc *vec, const int32_t *active, int nvec, hipStream_t s)
{
    switch (r.nv) {
    case 1: hipLaunchKernelGGL(k_red_finalize<1>, dim3(nvec), dim3(1024), 0, s, r, vec, active); break;
    case 2: hipLaunchKernelGGL(k_red_finalize<2>, dim3(nvec), dim3(1024), 0, s, r, vec, active); break;
    case 3: hipLaunchKernelGGL(k_red_finalize<3>, dim3(nvec), dim3(1024), 0, s, r, vec, active); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blas(int op, int prec, const BlasArgs &a, int block, hipStream_t s)
{
    switch (prec) {
    case P_F64: return launch_blas_t<P_F64>(op, a, block, s);
    case P_F32: return launch_blas_t<P_F32>(op, a, block, s);
    case P_F16: return launch_blas_t<P_F16>(op, a, block, s);
    case P_BF16: return launch_blas_t<P_BF16>(op, a, block, s);
    }
    return hipErrorInvalidValue;
}

template <int PD>
static hipError_t launch_convert_d(int ps, const BlasArgs &a, int block, hipStream_t s)
{
    dim3 g(a.nblocks), b(block);
    switch (ps) {
    case P_F64: hipLaunchKernelGGL((k_convert<PD, P_F64>), g, b, 0, s, a); break;
    case P_F32: hipLaunchKernelGGL((k_convert<PD, P_F32>), g, b, 0, s, a); break;
    case P_F16: hipLaunchKernelGGL((k_convert<PD, P_F16>), g, b, 0, s, a); break;
    case P_BF16: hipLaunchKernelGGL((k_convert<PD, P_BF16>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(int pd, int ps, const BlasArgs &a, int block, hipStream_t s)
{
    switch (pd) {
    case P_F64: return launch_convert_d<P_F64>(ps, a, block, s);
    case P_F32: return launch_convert_d<P_F32>(ps, a, block, s);
    case P_F16: return launch_convert_d<P_F16>(ps, a, block, s);
    case P_BF16: return launch_convert_d<P_BF16>(ps, a, block, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace wl
