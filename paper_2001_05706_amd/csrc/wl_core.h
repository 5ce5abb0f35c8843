// wl_core.h -- storage formats, packed loads/stores and the per-site Wilson
// hopping term for gfx950.
//
// Everything here is __host__ __device__ so that the same arithmetic can be
// exercised by a host build in the tests; the GPU kernels in *.hip include it.
//
// Packed layouts (structure of arrays, one parity per field):
//   A "vector" is one right-hand side of one system on the Vh = V/2 sites of
//   one parity, checkerboard index cb = s >> 1 (s the lexicographic site).
//   Its 24 reals are split into 16-byte (or 8-byte) chunks; chunk c of site cb
//   lives at  base[(site_off * NCHUNK) + c * stride + cb]  in units of the
//   chunk type, so that consecutive lanes (sites) read consecutive chunks.
//   FP64: 12 x double2          (one complex per chunk)
//   FP32:  6 x float4           (two complex per chunk)
//   FP16 / BF16: 3 x uint4      (four complex per chunk, value / site norm)
//                + one float norm per site (max |v| over the 24 reals)
//   Links of one system: [parity][mu][chunk][stride] with
//   FP64 recon-18: 9 x double2, FP64 recon-12: 6 x double2,
//   FP32 recon-18: 9 x float2,  FP32 recon-12: 3 x float4,
//   FP16 / BF16 recon-12: 3 x uint2 (two complex per chunk, no norm: |U_ij| <= 1).
//   Recon-12 keeps rows 0 and 1; row 2 = conj(row0 x row1), exact for SU(3).
//
// Spin-colour order of the 24 reals: v[2*(3*spin + colour) + {0: re, 1: im}],
// DeGrand-Rossi gamma basis.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WL_HD __host__ __device__ __forceinline__

namespace wl {

enum { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

// ------------------------------------------------------------------ complex

template <class T>
struct cpx {
    T re, im;
};

template <class T> WL_HD cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> WL_HD cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
// a + i b, a - i b
template <class T> WL_HD cpx<T> cadd_i(cpx<T> a, cpx<T> b) { return {a.re - b.im, a.im + b.re}; }
template <class T> WL_HD cpx<T> csub_i(cpx<T> a, cpx<T> b) { return {a.re + b.im, a.im - b.re}; }

// fused multiply-add, one rounding (IEEE fma on host and device)
WL_HD float fmadd(float a, float b, float c) { return fmaf(a, b, c); }
WL_HD double fmadd(double a, double b, double c) { return fma(a, b, c); }

// complex products with their fused multiply-adds written out: left to the
// compiler, which of the two products gets fused can differ between kernels
// built from the same source, and every launch variant must round alike
template <class T> WL_HD cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {fmadd(a.re, b.re, -(a.im * b.im)), fmadd(a.re, b.im, a.im * b.re)};
}
// conj(a) * b
template <class T> WL_HD cpx<T> cjmul(cpx<T> a, cpx<T> b)
{
    return {fmadd(a.re, b.re, a.im * b.im), fmadd(a.re, b.im, -(a.im * b.re))};
}

// ------------------------------------------------------------------ half / bf16

WL_HD float bf16_to_float(uint16_t h)
{
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)h << 16;
    return c.f;
}

// round to nearest even (inputs are finite and |x| <= 1 here)
WL_HD uint16_t float_to_bf16(float f)
{
    union { uint32_t u; float f; } c;
    c.f = f;
    uint32_t u = c.u;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

WL_HD float f16_to_float(uint16_t h)
{
    union { uint16_t u; _Float16 f; } c;
    c.u = h;
    return (float)c.f;
}

WL_HD uint16_t float_to_f16(float f)
{
    union { uint16_t u; _Float16 f; } c;
    c.f = (_Float16)f;  // round to nearest even
    return c.u;
}

template <int P> WL_HD float lo16_to_float(uint32_t w)
{
    return P == P_F16 ? f16_to_float((uint16_t)(w & 0xFFFFu)) : bf16_to_float((uint16_t)(w & 0xFFFFu));
}
template <int P> WL_HD float hi16_to_float(uint32_t w)
{
    return P == P_F16 ? f16_to_float((uint16_t)(w >> 16)) : bf16_to_float((uint16_t)(w >> 16));
}
// low (H = 0) or high (H = 1) half of a packed word as FP32
template <int P, int H> WL_HD float half_part(uint32_t w)
{
    if constexpr (P == P_F16) return H ? hi16_to_float<P>(w) : lo16_to_float<P>(w);
    union { uint32_t u; float f; } c;
    c.u = H ? (w & 0xFFFF0000u) : (w << 16);
    return c.f;
}

template <int P> WL_HD uint32_t pack2(float lo, float hi)
{
    uint32_t a = P == P_F16 ? float_to_f16(lo) : float_to_bf16(lo);
    uint32_t b = P == P_F16 ? float_to_f16(hi) : float_to_bf16(hi);
    return a | (b << 16);
}

// the FP16 number nearest to an FP64 one (a single rounding, to nearest even)
WL_HD uint16_t double_to_f16(double d)
{
    union { uint16_t u; _Float16 f; } c;
    c.f = (_Float16)d;
    return c.u;
}

// Two FP64 values (links, clover entries) in half precision: FP16 rounds each
// once from FP64; BF16 rounds to FP32, then to BF16 on its bits.
template <int P> WL_HD uint32_t pack2_d(double lo, double hi)
{
    if constexpr (P == P_F16) return (uint32_t)double_to_f16(lo) | ((uint32_t)double_to_f16(hi) << 16);
    return pack2<P>((float)lo, (float)hi);
}

// ------------------------------------------------------------------ storage traits

template <int P> struct SpinorFmt;
template <> struct SpinorFmt<P_F64> {
    using real = double;
    using chunk = double2;
    static constexpr int nchunk = 12;
    static constexpr bool has_norm = false;
    static constexpr int site_bytes = 192;
};
template <> struct SpinorFmt<P_F32> {
    using real = float;
    using chunk = float4;
    static constexpr int nchunk = 6;
    static constexpr bool has_norm = false;
    static constexpr int site_bytes = 96;
};
template <> struct SpinorFmt<P_F16> {
    using real = float;
    using chunk = uint4;
    static constexpr int nchunk = 3;
    static constexpr bool has_norm = true;
    static constexpr int site_bytes = 52;  // 48 + 4-byte norm
};
template <> struct SpinorFmt<P_BF16> : SpinorFmt<P_F16> {};

template <int P, int R> struct LinkFmt;
template <> struct LinkFmt<P_F64, 18> { using chunk = double2; static constexpr int nchunk = 9; static constexpr int bytes = 144; };
template <> struct LinkFmt<P_F64, 12> { using chunk = double2; static constexpr int nchunk = 6; static constexpr int bytes = 96; };
template <> struct LinkFmt<P_F32, 18> { using chunk = float2; static constexpr int nchunk = 9; static constexpr int bytes = 72; };
template <> struct LinkFmt<P_F32, 12> { using chunk = float4; static constexpr int nchunk = 3; static constexpr int bytes = 48; };
template <> struct LinkFmt<P_F16, 12> { using chunk = uint2; static constexpr int nchunk = 3; static constexpr int bytes = 24; };
template <> struct LinkFmt<P_BF16, 12> { using chunk = uint2; static constexpr int nchunk = 3; static constexpr int bytes = 24; };

// ------------------------------------------------------------------ memory access

// loads of streamed-once data (links) with the non-temporal hint, through
// native clang vector types (the HIP vector structs are not accepted by the builtin)
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t nt_u2 __attribute__((ext_vector_type(2)));
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));

// Field data lives in global memory: on the device the access helpers use
// pointers in the global address space, so that every load and store is a
// global instruction (a generic pointer read from a descriptor would compile to
// flat instructions, which also occupy the LDS counter the waits test).
#if defined(__HIP_DEVICE_COMPILE__)
#define WL_G __attribute__((address_space(1)))
#define WL_NT_LOAD(VT, p) __builtin_nontemporal_load((const WL_G VT *)(p))
#define WL_NT_STORE(VT, v, p) __builtin_nontemporal_store((v), (WL_G VT *)(p))
#else
#define WL_G
#define WL_NT_LOAD(VT, p) (*(const VT *)(p))
#define WL_NT_STORE(VT, v, p) (*(VT *)(p) = (v))
#endif

// stores of written-once data (a kernel's output field), plain or with the
// non-temporal hint
template <bool NT> WL_HD void st_out(WL_G double2 *p, double2 v)
{
    if constexpr (NT) WL_NT_STORE(nt_d2, (nt_d2{v.x, v.y}), p);
    else *p = v;
}
template <bool NT> WL_HD void st_out(WL_G float4 *p, float4 v)
{
    if constexpr (NT) WL_NT_STORE(nt_f4, (nt_f4{v.x, v.y, v.z, v.w}), p);
    else *p = v;
}
template <bool NT> WL_HD void st_out(WL_G uint4 *p, uint4 v)
{
    if constexpr (NT) WL_NT_STORE(nt_u4, (nt_u4{v.x, v.y, v.z, v.w}), p);
    else *p = v;
}
template <bool NT> WL_HD void st_out(WL_G float *p, float v)
{
    if constexpr (NT) WL_NT_STORE(float, v, p);
    else *p = v;
}

WL_HD double2 ld_stream(const WL_G double2 *p)
{
    const nt_d2 v = WL_NT_LOAD(nt_d2, p);
    return double2{v.x, v.y};
}
WL_HD float2 ld_stream(const WL_G float2 *p)
{
    const nt_f2 v = WL_NT_LOAD(nt_f2, p);
    return float2{v.x, v.y};
}
WL_HD float4 ld_stream(const WL_G float4 *p)
{
    const nt_f4 v = WL_NT_LOAD(nt_f4, p);
    return float4{v.x, v.y, v.z, v.w};
}
WL_HD uint2 ld_stream(const WL_G uint2 *p)
{
    const nt_u2 v = WL_NT_LOAD(nt_u2, p);
    return uint2{v.x, v.y};
}
WL_HD uint4 ld_stream(const WL_G uint4 *p)
{
    const nt_u4 v = WL_NT_LOAD(nt_u4, p);
    return uint4{v.x, v.y, v.z, v.w};
}
WL_HD float ld_stream(const WL_G float *p) { return WL_NT_LOAD(float, p); }

// load of a field element: plain, or with the non-temporal hint for fields
// read once per launch
template <bool NT, class CH> WL_HD CH ld_field(const WL_G CH *p)
{
    if constexpr (NT)
        return ld_stream(p);
    else
        return *p;
}

// The address of a row base held in scalar registers.  `base` must be the
// same in every lane of the wave (every kernel here takes its field bases from
// per-block or per-wave descriptors); the base is read from the first lane, so
// the compiler keeps one scalar base per row instead of folding the lane
// offset into a 64-bit vector address shared by the rows.
WL_HD uintptr_t uniform_addr(uintptr_t a)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return ((uintptr_t)hi << 32) | lo;
#else
    return a;
#endif
}

// Element `cb` of chunk row `c`: a uniform row base (scalar registers) plus a
// 32-bit lane offset, so each load is one global instruction with a scalar base
// and a 32-bit vector offset, and needs no 64-bit vector address arithmetic.
template <class CH> WL_HD const WL_G CH *row_elem(const void *base, int c, int stride, int cb)
{
    const WL_G char *row =
        (const WL_G char *)uniform_addr((uintptr_t)base + (size_t)c * (size_t)stride * sizeof(CH));
    return (const WL_G CH *)(row + (uint32_t)((uint32_t)cb * (uint32_t)sizeof(CH)));
}
template <class CH> WL_HD WL_G CH *row_elem(void *base, int c, int stride, int cb)
{
    WL_G char *row = (WL_G char *)uniform_addr((uintptr_t)base + (size_t)c * (size_t)stride * sizeof(CH));
    return (WL_G CH *)(row + (uint32_t)((uint32_t)cb * (uint32_t)sizeof(CH)));
}

// 24 reals of one site of one vector.  base points at chunk 0 of the vector.
// NT: non-temporal loads (a field streamed once by the launch).
template <int P, bool NT = false>
WL_HD void load_spinor(const void *base, const float *norm, int stride, int cb,
                       typename SpinorFmt<P>::real v[24])
{
    using F = SpinorFmt<P>;
    using CH = typename F::chunk;
    if constexpr (P == P_F64) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double2 w = ld_field<NT>(row_elem<CH>(base, c, stride, cb));
            v[2 * c] = w.x;
            v[2 * c + 1] = w.y;
        }
    } else if constexpr (P == P_F32) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            float4 w = ld_field<NT>(row_elem<CH>(base, c, stride, cb));
            v[4 * c] = w.x;
            v[4 * c + 1] = w.y;
            v[4 * c + 2] = w.z;
            v[4 * c + 3] = w.w;
        }
    } else {
        const float nrm = ld_field<NT>(row_elem<float>(norm, 0, 0, cb));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uint4 w = ld_field<NT>(row_elem<CH>(base, c, stride, cb));
            uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[8 * c + 2 * k] = lo16_to_float<P>(q[k]) * nrm;
                v[8 * c + 2 * k + 1] = hi16_to_float<P>(q[k]) * nrm;
            }
        }
    }
}

// The 12 packed complex words of a half-precision site and its norm.
template <int P, bool NT = false>
WL_HD void load_spinor_words(const void *base, const float *norm, int stride, int cb, uint32_t q[12], float *nrm)
{
    using CH = typename SpinorFmt<P>::chunk;
    *nrm = ld_field<NT>(row_elem<float>(norm, 0, 0, cb));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        uint4 w = ld_field<NT>(row_elem<CH>(base, c, stride, cb));
        q[4 * c] = w.x;
        q[4 * c + 1] = w.y;
        q[4 * c + 2] = w.z;
        q[4 * c + 3] = w.w;
    }
}

// The 24 reals of a site before its half-precision norm is applied, and that
// norm in *nrm (FP64/FP32: the values themselves and 1).  A caller folds the
// norm into a per-site coefficient; FP16 values then enter mixed-precision fmas
// directly.
template <int P, bool NT = false>
WL_HD void load_spinor_raw(const void *base, const float *norm, int stride, int cb,
                           typename SpinorFmt<P>::real v[24], typename SpinorFmt<P>::real *nrm)
{
    if constexpr (P == P_F64 || P == P_F32) {
        load_spinor<P, NT>(base, norm, stride, cb, v);
        *nrm = 1;
    } else {
        uint32_t q[12];
        float n;
        load_spinor_words<P, NT>(base, norm, stride, cb, q, &n);
        *nrm = n;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            v[2 * k] = half_part<P, 0>(q[k]);
            v[2 * k + 1] = half_part<P, 1>(q[k]);
        }
    }
}

template <int P, bool NT = false>
WL_HD void store_spinor(void *base, float *norm, int stride, int cb, const typename SpinorFmt<P>::real v[24])
{
    using F = SpinorFmt<P>;
    typename F::chunk *b = (typename F::chunk *)base;
    if constexpr (P == P_F64) {
#pragma unroll
        for (int c = 0; c < 12; ++c) st_out<NT>(row_elem<double2>(b, c, stride, cb), double2{v[2 * c], v[2 * c + 1]});
    } else if constexpr (P == P_F32) {
#pragma unroll
        for (int c = 0; c < 6; ++c)
            st_out<NT>(row_elem<float4>(b, c, stride, cb), float4{v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]});
    } else {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf(v[k]));
        // a zero site stores zeros and a zero norm (point sources are zero almost everywhere).
        // Stored value: v * inv with inv = 1/m correctly rounded; for FP16 the multiply
        // and the conversion compile to one mixed-precision fma (v_fma_mixlo/hi_f16), so
        // the exact product is rounded once to nearest even; BF16 rounds the FP32
        // product to nearest even on its bits.
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        st_out<NT>(row_elem<float>(norm, 0, 0, cb), m);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uint32_t q[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = pack2<P>(v[8 * c + 2 * k] * inv, v[8 * c + 2 * k + 1] * inv);
            st_out<NT>(row_elem<uint4>(b, c, stride, cb), uint4{q[0], q[1], q[2], q[3]});
        }
    }
}

// One link as a 3x3 complex matrix.  base points at chunk 0 of the (parity, mu) block.
// Link element load: non-temporal (NT) when each link is used once per launch,
// plain when other right-hand sides of the launch re-read it from L2.
template <bool NT, class CH> WL_HD CH ld_link(const WL_G CH *p)
{
    if constexpr (NT)
        return ld_stream(p);
    else
        return *p;
}

template <int P, int R, class T, bool NT = true>
WL_HD void load_link(const void *base, int stride, int cb, cpx<T> u[3][3])
{
    if constexpr (P == P_F64) {
#pragma unroll
        for (int k = 0; k < (R == 18 ? 9 : 6); ++k) {
            double2 w = ld_link<NT>(row_elem<double2>(base, k, stride, cb));
            u[k / 3][k % 3] = cpx<T>{(T)w.x, (T)w.y};
        }
    } else if constexpr (P == P_F32 && R == 18) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            float2 w = ld_link<NT>(row_elem<float2>(base, k, stride, cb));
            u[k / 3][k % 3] = cpx<T>{(T)w.x, (T)w.y};
        }
    } else if constexpr (P == P_F32) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float4 w = ld_link<NT>(row_elem<float4>(base, c, stride, cb));
            const int k = 2 * c;
            u[k / 3][k % 3] = cpx<T>{(T)w.x, (T)w.y};
            u[(k + 1) / 3][(k + 1) % 3] = cpx<T>{(T)w.z, (T)w.w};
        }
    } else {
        // FP16/BF16 recon-12: the first four complex entries in one 16-byte
        // row (the first two 8-byte chunk rows of the block), the last two in
        // the third 8-byte row: two loads per link instead of three
        const uint4 w01 = ld_link<NT>(row_elem<uint4>(base, 0, stride, cb));
        const uint2 w2 = ld_link<NT>(row_elem<uint2>(base, 2, stride, cb));
        const uint32_t q[6] = {w01.x, w01.y, w01.z, w01.w, w2.x, w2.y};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            u[k / 3][k % 3] = cpx<T>{(T)lo16_to_float<P>(q[k]), (T)hi16_to_float<P>(q[k])};
    }
    if constexpr (R == 12) {
        // row2 = conj(row0 x row1): u2k = conj(u0i u1j - u0j u1i), (k, i, j) cyclic
        auto cross = [](cpx<T> a, cpx<T> b, cpx<T> c, cpx<T> d) -> cpx<T> {
            if constexpr (sizeof(T) == 4) {
                // FP32 arithmetic: chains of fused multiply-adds (fewer instructions);
                // each chain opens with an fma on zero so that half-precision
                // operands enter the mixed-precision fma without a conversion
                T re = fmadd(a.re, b.re, T(0));
                re = fmadd(-a.im, b.im, re);
                re = fmadd(-c.re, d.re, re);
                re = fmadd(c.im, d.im, re);
                T im = fmadd(c.re, d.im, T(0));
                im = fmadd(c.im, d.re, im);
                im = fmadd(-a.re, b.im, im);
                im = fmadd(-a.im, b.re, im);
                return {re, im};
            } else {
                // FP64 (memory-bound): independent products keep fewer registers
                // live; conj(a b - c d), fused multiply-adds written out
                const cpx<T> ab = cmul(a, b), cd = cmul(c, d);
                return {ab.re - cd.re, cd.im - ab.im};
            }
        };
        u[2][0] = cross(u[0][1], u[1][2], u[0][2], u[1][1]);
        u[2][1] = cross(u[0][2], u[1][0], u[0][0], u[1][2]);
        u[2][2] = cross(u[0][0], u[1][1], u[0][1], u[1][0]);
    }
}

template <int P, int R>
WL_HD void store_link(void *base, int stride, int cb, const double u[18] /* row-major complex */)
{
    using F = LinkFmt<P, R>;
    typename F::chunk *b = (typename F::chunk *)base;
    if constexpr (P == P_F64) {
        for (int k = 0; k < (R == 18 ? 9 : 6); ++k) b[(size_t)k * stride + cb] = double2{u[2 * k], u[2 * k + 1]};
    } else if constexpr (P == P_F32 && R == 18) {
        for (int k = 0; k < 9; ++k) b[(size_t)k * stride + cb] = float2{(float)u[2 * k], (float)u[2 * k + 1]};
    } else if constexpr (P == P_F32) {
        for (int c = 0; c < 3; ++c)
            b[(size_t)c * stride + cb] = float4{(float)u[4 * c], (float)u[4 * c + 1], (float)u[4 * c + 2], (float)u[4 * c + 3]};
    } else {
        // entries 0-3 as one 16-byte row over chunk rows 0 and 1, entries 4-5 in row 2
        uint4 *r01 = (uint4 *)base;
        r01[cb] = uint4{pack2_d<P>(u[0], u[1]), pack2_d<P>(u[2], u[3]), pack2_d<P>(u[4], u[5]),
                        pack2_d<P>(u[6], u[7])};
        b[(size_t)2 * stride + cb] = uint2{pack2_d<P>(u[8], u[9]), pack2_d<P>(u[10], u[11])};
    }
}

// ------------------------------------------------------------------ geometry

// Per-system lattice description (lives in device memory; read with scalar loads).
struct SysDesc {
    int32_t L[4];
    int32_t Lxh;         // Lx / 2
    int32_t Vh;          // sites per parity
    int32_t stride;      // chunk stride of one vector (>= Vh, multiple of 64)
    int32_t tap;         // 1: antiperiodic in t
    int32_t gstride;     // chunk stride of the packed links (== stride)
    int32_t pad_;
    const void *gauge;   // packed links of the precision used by the launch
    const void *clov;    // packed clover term A (null: Wilson system), [parity][chunk][stride]
    const void *clovinv; // packed A^{-1}
    double inv_lxh, inv_l1, inv_l2;  // 1/Lxh, 1/L[1], 1/L[2] for the coordinate divisions (set_divisors)
};

// the reciprocals cb_coords divides by (host side, once per geometry)
inline void set_divisors(SysDesc &d)
{
    d.inv_lxh = 1.0 / d.Lxh;
    d.inv_l1 = 1.0 / d.L[1];
    d.inv_l2 = 1.0 / d.L[2];
}

// floor(n / d) for 0 <= n < 2^26 and 1 <= d <= 2^19, given inv = 1/d rounded to
// FP64: n * inv is within 2^-26 of n/d, so adding 2^-20 lifts an exact quotient
// clear of the truncation and stays below the next integer, which is at least
// 1/d >= 2^-19 away (three FP64 instructions instead of an integer division)
WL_HD int idiv(int n, double inv) { return (int)fma((double)n, inv, 0x1p-20); }

// ------------------------------------------------------------------ clover term
//
// A(x) = 1 + i kappa c_sw sum_{m<n} s_mn F_mn(x) commutes with g5, so in the
// DeGrand-Rossi basis it is two Hermitian 6x6 blocks: block b acts on spins
// 2b, 2b+1 (all colours), i.e. on the 12 reals o[12b .. 12b+11].  A block is
// packed as 36 reals: the 6 real diagonal entries, then the 15 entries above
// the diagonal in row-major order as (re, im).  FP64 stores 36 double2 rows per
// site, FP32 18 float4 rows, FP16 9 uint4 rows of 8 halves (the 72 reals of the
// two blocks in order; FP16 and BF16 launches read this copy).
template <int P> struct CloverFmt {
    using chunk = float4;
    static constexpr int nchunk = 18;
};
template <> struct CloverFmt<P_F64> {
    using chunk = double2;
    static constexpr int nchunk = 36;
};
template <> struct CloverFmt<P_F16> {
    using chunk = uint4;
    static constexpr int nchunk = 9;
};

// the copy of the clover term a launch of storage precision P reads
template <int P> constexpr int clover_prec() { return P == P_F64 ? P_F64 : P == P_F32 ? P_F32 : P_F16; }

// packed index of entry (i, j), i < j, of a 6x6 block
WL_HD int clov_upper(int i, int j) { return 6 + 2 * (i * 6 - i * (i + 1) / 2 + (j - i - 1)); }

// o <- A o (or A^{-1} o for the inverse field) at site cb; base is the parity's chunk 0
template <int P, class T>
WL_HD void clover_apply(const void *base, int stride, int cb, T o[24])
{
    using CF = CloverFmt<P>;
    uint32_t h[36];  // FP16: the site's 72 halves, two per word
    if constexpr (P == P_F16) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const uint4 w = *row_elem<uint4>(base, c, stride, cb);
            h[4 * c] = w.x;
            h[4 * c + 1] = w.y;
            h[4 * c + 2] = w.z;
            h[4 * c + 3] = w.w;
        }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        T m[36];
        if constexpr (P == P_F16) {
#pragma unroll
            for (int k = 0; k < 36; ++k) {
                const int e = 36 * b + k;
                m[k] = (T)(e & 1 ? hi16_to_float<P_F16>(h[e >> 1]) : lo16_to_float<P_F16>(h[e >> 1]));
            }
        } else if constexpr (P == P_F64) {
#pragma unroll
            for (int c = 0; c < 18; ++c) {
                const double2 w = *row_elem<double2>(base, 18 * b + c, stride, cb);
                m[2 * c] = (T)w.x;
                m[2 * c + 1] = (T)w.y;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const float4 w = *row_elem<typename CF::chunk>(base, 9 * b + c, stride, cb);
                m[4 * c] = (T)w.x;
                m[4 * c + 1] = (T)w.y;
                m[4 * c + 2] = (T)w.z;
                m[4 * c + 3] = (T)w.w;
            }
        }
        T xr[6], xi[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            xr[k] = o[12 * b + 2 * k];
            xi[k] = o[12 * b + 2 * k + 1];
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            T yr = m[i] * xr[i], yi = m[i] * xi[i];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                if (j == i) continue;
                // M_ij = (re, im) for i < j; M_ij = conj(M_ji) for i > j
                const int u = i < j ? clov_upper(i, j) : clov_upper(j, i);
                const T mr = m[u], mi = i < j ? m[u + 1] : -m[u + 1];
                // fused multiply-adds written out (every launch variant rounds alike)
                yr = fmadd(mr, xr[j], yr);
                yr = fmadd(-mi, xi[j], yr);
                yi = fmadd(mr, xi[j], yi);
                yi = fmadd(mi, xr[j], yi);
            }
            o[12 * b + 2 * i] = yr;
            o[12 * b + 2 * i + 1] = yi;
        }
    }
}

// base of parity `par` of a packed clover field
template <int P> WL_HD const void *clover_parity(const void *f, int par, int stride)
{
    return (const char *)f + (size_t)par * CloverFmt<P>::nchunk * stride * sizeof(typename CloverFmt<P>::chunk);
}

// site coordinates from checkerboard index and parity
struct Site {
    int x, y, z, t;
};

WL_HD Site cb_coords(const SysDesc &d, int cb, int parity)
{
    Site s;
    const int r0 = idiv(cb, d.inv_lxh);  // cb = xh + Lxh (y + L1 (z + L2 t))
    const int xh = cb - r0 * d.Lxh;
    const int r1 = idiv(r0, d.inv_l1);
    s.y = r0 - r1 * d.L[1];
    s.t = idiv(r1, d.inv_l2);
    s.z = r1 - s.t * d.L[2];
    s.x = 2 * xh + ((s.y + s.z + s.t + parity) & 1);
    return s;
}

// ------------------------------------------------------------------ half-spinor algebra
//
// For P = 1 + sg * gamma_mu (sg = -1 forward hop of H, +1 backward; swapped for
// H^dagger) the 4-spinor P psi is fixed by two spin components h0, h1:
//   mu=x: h0 = p0 + sg i p3, h1 = p1 + sg i p2;   rows 2,3 = -sg i h1, -sg i h0
//   mu=y: h0 = p0 - sg p3,   h1 = p1 + sg p2;     rows 2,3 =  sg h1,  -sg h0
//   mu=z: h0 = p0 + sg i p2, h1 = p1 - sg i p3;   rows 2,3 = -sg i h0,  sg i h1
//   mu=t: h0 = p0 + sg p2,   h1 = p1 + sg p3;     rows 2,3 =  sg h0,   sg h1
// (from the DeGrand-Rossi matrices; 12 flop per projection, 24 per reconstruction)

template <int MU, int SG, class T>
WL_HD void project(const T v[24], cpx<T> h0[3], cpx<T> h1[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<T> p0{v[2 * (0 + c)], v[2 * (0 + c) + 1]};
        cpx<T> p1{v[2 * (3 + c)], v[2 * (3 + c) + 1]};
        cpx<T> p2{v[2 * (6 + c)], v[2 * (6 + c) + 1]};
        cpx<T> p3{v[2 * (9 + c)], v[2 * (9 + c) + 1]};
        if constexpr (MU == 0) {
            h0[c] = SG > 0 ? cadd_i(p0, p3) : csub_i(p0, p3);
            h1[c] = SG > 0 ? cadd_i(p1, p2) : csub_i(p1, p2);
        } else if constexpr (MU == 1) {
            h0[c] = SG > 0 ? csub(p0, p3) : cadd(p0, p3);
            h1[c] = SG > 0 ? cadd(p1, p2) : csub(p1, p2);
        } else if constexpr (MU == 2) {
            h0[c] = SG > 0 ? cadd_i(p0, p2) : csub_i(p0, p2);
            h1[c] = SG > 0 ? csub_i(p1, p3) : cadd_i(p1, p3);
        } else {
            h0[c] = SG > 0 ? cadd(p0, p2) : csub(p0, p2);
            h1[c] = SG > 0 ? cadd(p1, p3) : csub(p1, p3);
        }
    }
}

// ---- half-precision projection straight from the packed words
//
// A half-precision spinor word holds one complex number (real part in the low
// 16 bits).  a_h + s b_h of two such halves is formed in FP32 without separate
// conversions: FP16 through one mixed-precision fma (a * 1 + (+-b), each half
// selected in place), BF16 by moving the half to the top of an FP32 word.

template <int P, int HA, int HB, bool NEG> WL_HD float half_sum(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (P == P_F16) {
        float d;
        // op_sel picks the half of each word, op_sel_hi marks sources 0 and 2 as FP16;
        // the 1.0 multiplier sits in a scalar register (an FP32 operand)
        if constexpr (NEG)
            asm("v_fma_mix_f32 %0, %1, %2, -%3 op_sel:[%4,0,%5] op_sel_hi:[1,0,1]"
                : "=v"(d) : "v"(a), "s"(1.0f), "v"(b), "i"(HA), "i"(HB));
        else
            asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[%4,0,%5] op_sel_hi:[1,0,1]"
                : "=v"(d) : "v"(a), "s"(1.0f), "v"(b), "i"(HA), "i"(HB));
        return d;
    }
#endif
    const float x = half_part<P, HA>(a), y = half_part<P, HB>(b);
    return NEG ? x - y : x + y;
}

// a + s b of two packed complex words, s = +1, -1, +i, -i (S = 0, 1, 2, 3)
template <int P, int S> WL_HD cpx<float> half_comb(uint32_t a, uint32_t b)
{
    if constexpr (S == 0) return {half_sum<P, 0, 0, false>(a, b), half_sum<P, 1, 1, false>(a, b)};
    if constexpr (S == 1) return {half_sum<P, 0, 0, true>(a, b), half_sum<P, 1, 1, true>(a, b)};
    // a + i b = (a.re - b.im, a.im + b.re);  a - i b = (a.re + b.im, a.im - b.re)
    if constexpr (S == 2) return {half_sum<P, 0, 1, true>(a, b), half_sum<P, 1, 0, false>(a, b)};
    return {half_sum<P, 0, 1, false>(a, b), half_sum<P, 1, 0, true>(a, b)};
}

// P psi (the projection of `project`) of a half-precision spinor given as its
// 12 packed complex words, site norm not applied
template <int P, int MU, int SG>
WL_HD void project_half(const uint32_t q[12], cpx<float> h0[3], cpx<float> h1[3])
{
    constexpr int ADD = 0, SUB = 1, ADD_I = 2, SUB_I = 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t p0 = q[0 + c], p1 = q[3 + c], p2 = q[6 + c], p3 = q[9 + c];
        if constexpr (MU == 0) {
            h0[c] = half_comb<P, (SG > 0 ? ADD_I : SUB_I)>(p0, p3);
            h1[c] = half_comb<P, (SG > 0 ? ADD_I : SUB_I)>(p1, p2);
        } else if constexpr (MU == 1) {
            h0[c] = half_comb<P, (SG > 0 ? SUB : ADD)>(p0, p3);
            h1[c] = half_comb<P, (SG > 0 ? ADD : SUB)>(p1, p2);
        } else if constexpr (MU == 2) {
            h0[c] = half_comb<P, (SG > 0 ? ADD_I : SUB_I)>(p0, p2);
            h1[c] = half_comb<P, (SG > 0 ? SUB_I : ADD_I)>(p1, p3);
        } else {
            h0[c] = half_comb<P, (SG > 0 ? ADD : SUB)>(p0, p2);
            h1[c] = half_comb<P, (SG > 0 ? ADD : SUB)>(p1, p3);
        }
    }
}

// acc += f P psi given U h0, U h1 of the unscaled projection: the factor f
// (site norm and boundary sign) rides on the accumulating fma
template <int MU, int SG, class T>
WL_HD void reconstruct_add_scaled(T acc[24], const cpx<T> g0[3], const cpx<T> g1[3], T f)
{
    const T nf = -f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[2 * (0 + c)] = fmadd(g0[c].re, f, acc[2 * (0 + c)]);
        acc[2 * (0 + c) + 1] = fmadd(g0[c].im, f, acc[2 * (0 + c) + 1]);
        acc[2 * (3 + c)] = fmadd(g1[c].re, f, acc[2 * (3 + c)]);
        acc[2 * (3 + c) + 1] = fmadd(g1[c].im, f, acc[2 * (3 + c) + 1]);
        // rows 2, 3 as in reconstruct_add, each term carrying +f or -f
        T r2re, r2im, r3re, r3im;
        T s2re, s2im, s3re, s3im;
        if constexpr (MU == 0) {
            r2re = g1[c].im; r2im = g1[c].re; s2re = SG > 0 ? f : nf; s2im = SG > 0 ? nf : f;
            r3re = g0[c].im; r3im = g0[c].re; s3re = SG > 0 ? f : nf; s3im = SG > 0 ? nf : f;
        } else if constexpr (MU == 1) {
            r2re = g1[c].re; r2im = g1[c].im; s2re = s2im = SG > 0 ? f : nf;
            r3re = g0[c].re; r3im = g0[c].im; s3re = s3im = SG > 0 ? nf : f;
        } else if constexpr (MU == 2) {
            r2re = g0[c].im; r2im = g0[c].re; s2re = SG > 0 ? f : nf; s2im = SG > 0 ? nf : f;
            r3re = g1[c].im; r3im = g1[c].re; s3re = SG > 0 ? nf : f; s3im = SG > 0 ? f : nf;
        } else {
            r2re = g0[c].re; r2im = g0[c].im; s2re = s2im = SG > 0 ? f : nf;
            r3re = g1[c].re; r3im = g1[c].im; s3re = s3im = SG > 0 ? f : nf;
        }
        acc[2 * (6 + c)] = fmadd(r2re, s2re, acc[2 * (6 + c)]);
        acc[2 * (6 + c) + 1] = fmadd(r2im, s2im, acc[2 * (6 + c) + 1]);
        acc[2 * (9 + c)] = fmadd(r3re, s3re, acc[2 * (9 + c)]);
        acc[2 * (9 + c) + 1] = fmadd(r3im, s3im, acc[2 * (9 + c) + 1]);
    }
}

// acc += P psi given U h0, U h1 (already multiplied by the link)
template <int MU, int SG, class T>
WL_HD void reconstruct_add(T acc[24], const cpx<T> g0[3], const cpx<T> g1[3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[2 * (0 + c)] += g0[c].re;
        acc[2 * (0 + c) + 1] += g0[c].im;
        acc[2 * (3 + c)] += g1[c].re;
        acc[2 * (3 + c) + 1] += g1[c].im;
        cpx<T> r2, r3;
        if constexpr (MU == 0) {
            // -sg i h1, -sg i h0 ; i(a+ib) = -b + ia
            r2 = SG > 0 ? cpx<T>{g1[c].im, -g1[c].re} : cpx<T>{-g1[c].im, g1[c].re};
            r3 = SG > 0 ? cpx<T>{g0[c].im, -g0[c].re} : cpx<T>{-g0[c].im, g0[c].re};
        } else if constexpr (MU == 1) {
            r2 = SG > 0 ? g1[c] : cpx<T>{-g1[c].re, -g1[c].im};
            r3 = SG > 0 ? cpx<T>{-g0[c].re, -g0[c].im} : g0[c];
        } else if constexpr (MU == 2) {
            r2 = SG > 0 ? cpx<T>{g0[c].im, -g0[c].re} : cpx<T>{-g0[c].im, g0[c].re};
            r3 = SG > 0 ? cpx<T>{-g1[c].im, g1[c].re} : cpx<T>{g1[c].im, -g1[c].re};
        } else {
            r2 = SG > 0 ? g0[c] : cpx<T>{-g0[c].re, -g0[c].im};
            r3 = SG > 0 ? g1[c] : cpx<T>{-g1[c].re, -g1[c].im};
        }
        acc[2 * (6 + c)] += r2.re;
        acc[2 * (6 + c) + 1] += r2.im;
        acc[2 * (9 + c)] += r3.re;
        acc[2 * (9 + c) + 1] += r3.im;
    }
}

// g = U h (ADJ = false) or U^dagger h (ADJ = true); in FP32 each output is a
// chain of fused multiply-adds
template <bool ADJ, class T>
WL_HD void su3_mul(const cpx<T> u[3][3], const cpx<T> h[3], cpx<T> g[3])
{
    if constexpr (sizeof(T) == 8) {
        // FP64 (memory-bound): independent products keep fewer registers live
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<T> s{0, 0};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const cpx<T> p = ADJ ? cjmul(u[b][a], h[b]) : cmul(u[a][b], h[b]);
                s.re += p.re;
                s.im += p.im;
            }
            g[a] = s;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T re = 0, im = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cpx<T> w = ADJ ? u[b][a] : u[a][b];
            // U h: (w.re h.re - w.im h.im, w.re h.im + w.im h.re); U^dagger: conj(w)
            const T wi = ADJ ? -w.im : w.im;
            // (the first term is an fma on zero as well: see load_link)
            re = fmadd(w.re, h[b].re, re);
            im = fmadd(w.re, h[b].im, im);
            re = fmadd(-wi, h[b].im, re);
            im = fmadd(wi, h[b].re, im);
        }
        g[a] = {re, im};
    }
}

// Everything the per-site hop needs.
struct HopSite {
    const void *in;       // input vector (opposite parity), chunk 0
    const float *in_norm; // FP16/BF16 norms of the input vector
    int stride;           // chunk stride of spinor vectors
    const void *gauge;    // packed links of the system: [parity][mu][chunk][gstride]
    int gstride;
    float scale = 1.0f;   // FP16/BF16: factor folded into the accumulation (unused otherwise)
};

// Neighbour of site s (checkerboard index cb) in direction +-mu: its
// checkerboard index, and whether the hop wraps the antiperiodic time boundary.
// In y, z and t the index moves by the direction's stride (Lxh, Lxh L1,
// Lxh L1 L2), wrapping at the lattice edge; in x the neighbour of x = 2 xh + o
// has half-index xh + o forwards and xh - (1 - o) backwards, wrapping in xh.
template <int MU, int DIR>
WL_HD int neighbour(const SysDesc &d, const Site &s, int cb, bool &flip)
{
    flip = false;
    if constexpr (MU == 0) {
        const int o = s.x & 1, xh = s.x >> 1;
        if constexpr (DIR > 0) return o ? (xh + 1 == d.Lxh ? cb - xh : cb + 1) : cb;
        return o ? cb : (xh == 0 ? cb + d.Lxh - 1 : cb - 1);
    } else {
        const int c = MU == 1 ? s.y : MU == 2 ? s.z : s.t;
        const int st = MU == 1 ? d.Lxh : MU == 2 ? d.Lxh * d.L[1] : d.Lxh * d.L[1] * d.L[2];
        const int span = (d.L[MU] - 1) * st;  // from the last slice back to the first
        if constexpr (DIR > 0) {
            const bool w = c + 1 == d.L[MU];
            if constexpr (MU == 3) flip = w && d.tap;
            return w ? cb - span : cb + st;
        } else {
            const bool w = c == 0;
            if constexpr (MU == 3) flip = w && d.tap;
            return w ? cb + span : cb - st;
        }
    }
}

// The spin projection of one neighbour spinor, and the factor its contribution
// carries: FP16/BF16 are projected straight from the packed words, the site
// norm and the boundary sign (and the hop coefficient a.scale) ride on the
// accumulating fma; FP64/FP32 take the boundary sign here and f = 1.
template <int SP, int MU, int SG, class T>
WL_HD T project_neighbour(const HopSite &a, int ncb, bool flip, cpx<T> h0[3], cpx<T> h1[3])
{
    if constexpr (SP == P_F16 || SP == P_BF16) {
        uint32_t q[12];
        T nrm;
        load_spinor_words<SP>(a.in, a.in_norm, a.stride, ncb, q, &nrm);
        project_half<SP, MU, SG>(q, h0, h1);
        return (flip ? -nrm : nrm) * (T)a.scale;
    } else {
        T v[24];
        load_spinor<SP>(a.in, nullptr, a.stride, ncb, v);
        project<MU, SG>(v, h0, h1);
        if (flip) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                h0[c] = {-h0[c].re, -h0[c].im};
                h1[c] = {-h1[c].re, -h1[c].im};
            }
        }
        return 1;
    }
}

// forward: U_mu(x) on this parity; backward: U_mu(x - mu)^dagger on the other parity
template <int GP, int R, int MU, int DIR, bool NT, class T>
WL_HD void hop_link(const HopSite &a, int parity, int cb, int ncb, cpx<T> u[3][3])
{
    constexpr int NCH = LinkFmt<GP, R>::nchunk;
    const int lpar = DIR > 0 ? parity : 1 - parity;
    const int lcb = DIR > 0 ? cb : ncb;
    const char *lbase = (const char *)a.gauge +
                        (size_t)((lpar * 4 + MU) * NCH) * a.gstride * sizeof(typename LinkFmt<GP, R>::chunk);
    load_link<GP, R, T, NT>(lbase, a.gstride, lcb, u);
}

// acc += f P (U h0, U h1)
template <int SP, int MU, int DIR, int SG, class T>
WL_HD void hop_accumulate(const cpx<T> u[3][3], const cpx<T> h0[3], const cpx<T> h1[3], T f, T acc[24])
{
    cpx<T> g0[3], g1[3];
    su3_mul<(DIR < 0), T>(u, h0, g0);
    su3_mul<(DIR < 0), T>(u, h1, g1);
    if constexpr (SP == P_F16 || SP == P_BF16)
        reconstruct_add_scaled<MU, SG>(acc, g0, g1, f);
    else
        reconstruct_add<MU, SG>(acc, g0, g1);
}

template <int SP, int GP, int R, int MU, int DIR, bool DAG, bool NT, class T>
WL_HD void hop_dir(const SysDesc &d, const HopSite &a, int parity, const Site &s, int cb, T acc[24])
{
    bool flip;
    const int ncb = neighbour<MU, DIR>(d, s, cb, flip);
    // forward hop carries 1 - gamma (sg = -1), backward 1 + gamma; adjoint swaps
    constexpr int SG = (DIR > 0) == DAG ? +1 : -1;
    cpx<T> h0[3], h1[3];
    const T f = project_neighbour<SP, MU, SG>(a, ncb, flip, h0, h1);
    cpx<T> u[3][3];
    hop_link<GP, R, MU, DIR, NT>(a, parity, cb, ncb, u);
    hop_accumulate<SP, MU, DIR, SG>(u, h0, h1, f, acc);
}

// The same direction for two right-hand sides of one system at one site: the
// neighbour index and the link (with its recon-12 row) are formed once.
template <int SP, int GP, int R, int MU, int DIR, bool DAG, bool NT, class T>
WL_HD void hop_dir2(const SysDesc &d, const HopSite &a0, const HopSite &a1, int parity, const Site &s, int cb,
                    T acc0[24], T acc1[24])
{
    bool flip;
    const int ncb = neighbour<MU, DIR>(d, s, cb, flip);
    constexpr int SG = (DIR > 0) == DAG ? +1 : -1;
    cpx<T> u[3][3];
    hop_link<GP, R, MU, DIR, NT>(a0, parity, cb, ncb, u);
    {
        cpx<T> h0[3], h1[3];
        const T f = project_neighbour<SP, MU, SG>(a0, ncb, flip, h0, h1);
        hop_accumulate<SP, MU, DIR, SG>(u, h0, h1, f, acc0);
    }
    {
        cpx<T> h0[3], h1[3];
        const T f = project_neighbour<SP, MU, SG>(a1, ncb, flip, h0, h1);
        hop_accumulate<SP, MU, DIR, SG>(u, h0, h1, f, acc1);
    }
}

// Keeps the compiler from hoisting the loads of later directions above this
// point: one direction pair's operands in flight per wave bounds the register
// footprint, and occupancy supplies the memory-level parallelism.
// The accumulator is passed through the fence as register operands so that the
// arithmetic of earlier directions completes before it (otherwise the loaded
// operands of every direction stay live until a combined tail).
template <class T> WL_HD void sched_fence(T acc[24])
{
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int k = 0; k < 24; ++k) asm volatile("" : "+v"(acc[k]));
    asm volatile("" ::: "memory");
#endif
}
#define WL_SCHED_FENCE() sched_fence(acc)

// acc = (H psi)(x) (or H^dagger) at output site cb of `parity`; psi is read on
// the other parity.  FENCE = number of directions whose operands may be in
// flight together (1, 2, 4 or 8); NT = non-temporal link loads.
template <int SP, int GP, int R, bool DAG, int FENCE = 2, bool NT = true, class T>
WL_HD void hop_site(const SysDesc &d, const HopSite &a, int parity, int cb, T acc[24])
{
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    const Site s = cb_coords(d, cb, parity);
    hop_dir<SP, GP, R, 0, +1, DAG, NT>(d, a, parity, s, cb, acc);
    if constexpr (FENCE == 1) WL_SCHED_FENCE();
    hop_dir<SP, GP, R, 0, -1, DAG, NT>(d, a, parity, s, cb, acc);
    if constexpr (FENCE <= 2) WL_SCHED_FENCE();
    hop_dir<SP, GP, R, 1, +1, DAG, NT>(d, a, parity, s, cb, acc);
    if constexpr (FENCE == 1) WL_SCHED_FENCE();
    hop_dir<SP, GP, R, 1, -1, DAG, NT>(d, a, parity, s, cb, acc);
    if constexpr (FENCE <= 4) WL_SCHED_FENCE();
    hop_dir<SP, GP, R, 2, +1, DAG, NT>(d, a, parity, s, cb, acc);
    if constexpr (FENCE == 1) WL_SCHED_FENCE();
    hop_dir<SP, GP, R, 2, -1, DAG, NT>(d, a, parity, s, cb, acc);
    if constexpr (FENCE <= 2) WL_SCHED_FENCE();
    hop_dir<SP, GP, R, 3, +1, DAG, NT>(d, a, parity, s, cb, acc);
    if constexpr (FENCE == 1) WL_SCHED_FENCE();
    hop_dir<SP, GP, R, 3, -1, DAG, NT>(d, a, parity, s, cb, acc);
    WL_SCHED_FENCE();
}

// acc0, acc1 = (H psi)(x) of two right-hand sides of one system (a0, a1 name
// their input vectors), one direction in flight at a time.
template <int SP, int GP, int R, bool DAG, bool NT = false, class T>
WL_HD void hop_site2(const SysDesc &d, const HopSite &a0, const HopSite &a1, int parity, int cb, T acc0[24],
                     T acc1[24])
{
#pragma unroll
    for (int k = 0; k < 24; ++k) acc0[k] = acc1[k] = 0;
    const Site s = cb_coords(d, cb, parity);
#define WL_DIR2(MU, DIR)                                                                  \
    hop_dir2<SP, GP, R, MU, DIR, DAG, NT>(d, a0, a1, parity, s, cb, acc0, acc1);          \
    sched_fence(acc0);                                                                    \
    sched_fence(acc1);
    WL_DIR2(0, +1)
    WL_DIR2(0, -1)
    WL_DIR2(1, +1)
    WL_DIR2(1, -1)
    WL_DIR2(2, +1)
    WL_DIR2(2, -1)
    WL_DIR2(3, +1)
    WL_DIR2(3, -1)
#undef WL_DIR2
}

}  // namespace wl
