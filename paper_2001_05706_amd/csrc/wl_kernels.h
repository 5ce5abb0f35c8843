// wl_kernels.h -- host-side launchers of the device kernels.
#pragma once

#include "wl_launch.h"

namespace wl {

struct BlasArgs {
    const SysDesc *sys;
    const VecDesc *vec;
    const BlkMap *map;
    const int32_t *active;
    int32_t nblocks;
    int32_t parity;    // parity of the fields (clover operations)
    void *f[6];
    float *fn[6];
    const double *s0;  // per-vector scalar (alpha or beta)
    const double *sc;  // scalar slots of the set (ScSlot), for complex scalars
    int32_t nvec;
    int32_t bcast;     // bit j: field j is one vector shared by every vector of the set
    int32_t one;       // the set holds one vector (its descriptors are at index 0)
    int32_t stream;    // solver-iteration kernels: fields read and written non-temporally
    RedSpec red;
};

constexpr int kMaxSys = 64;  // systems per set (canonical pointers travel by value)

struct PackArgs {
    const SysDesc *sys;
    const VecDesc *vec;
    const BlkMap *map;
    int32_t nblocks;
    int32_t parity;
    void *f;
    float *fn;
    const double *canon[kMaxSys];  // per system: canonical fields of all its rhs
};

// hop.hip
// var selects a launch variant (0 .. hop_variants(prec)-1, see hop.hip); clov
// selects the instantiation with the clover epilogue; with events e0/e1 the
// dispatch records them at the kernel's start and end
hipError_t launch_hop(int prec, int recon, bool dag, bool clov, int var, const HopArgs &a, int block, hipStream_t s,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
int hop_variants(int prec);  // launch variants available for a storage precision

// blas.hip -- all operate on the vectors of one set through its block map
enum BlasOp {
    BL_CG_UPDATE = 0,  // x += alpha p; r -= alpha q; |r|^2          f = {x, p, r, q}, s0 = alpha
    BL_XPAY = 1,       // p = s + beta p                             f = {p, s},       s0 = beta
    BL_ACCUM = 2,      // y(F64) += x; x = 0                         f = {y, x}
    BL_NORM2 = 3,      // |x|^2                                      f = {x}
    BL_ZERO = 4,       // x = 0                                      f = {x}
    BL_COPY = 5,       // y = x                                      f = {y, x}
    BL_FILL = 6,       // x = deterministic pattern (benchmark operands)  f = {x}
    BL_SCALE_RSQRT = 7,// x *= 1/sqrt(s0[v])                         f = {x}
    // BiCGStab (complex scalars from the slots):
    BL_BICG_P = 8,     // p = r + beta (p - omega v), beta = (rho/rho_prev)(alpha/omega)   f = {p, r, v}
    BL_BICG_S = 9,     // s = r - alpha v                                                   f = {s, r, v}
    BL_BICG_XR = 10,   // x += alpha p + omega s; r = s - omega t; <rhat, r>, |r|^2         f = {x, p, s, r, t, rhat}
    BL_CDOT = 11,      // <a, b>                                                            f = {a, b}
    BL_G5COPY = 12,    // y = g5 x                                                          f = {y, x}
    BL_CLOV_INV = 13,  // y = A^{-1} x on parity `parity` (clover systems; a copy otherwise)  f = {y, x}
    // deflation and block operations (single-system sets; complex scalars from s0):
    BL_CAXPY = 14,     // y += z x, z = (s0[2v], s0[2v+1])                                  f = {y, x}
    BL_CAXPY_G5 = 15,  // y += z g5 x                                                       f = {y, x}
    BL_ROT = 16,       // y_v = sum_j T[j + nvec v] x_j, T complex (s0)                      f = {y, x}
    // CGNR iteration with the solution update moved into the direction update:
    BL_R_UPDATE = 17,  // r -= alpha q; |r|^2                                               f = {r, q},    s0 = alpha
    BL_XPAY_X = 18,    // x += alpha p; p = s + beta p (alpha from its slot)                  f = {p, s, x}, s0 = beta
};
hipError_t launch_blas(int op, int prec, const BlasArgs &a, int block, hipStream_t s);
// fixed-order sum of each active vector's block partials and the reduction's finishing step
hipError_t launch_red_finalize(const RedSpec &r, const VecDesc *vec, const int32_t *active, int nvec, hipStream_t s);
// k deferred |r|^2 rows (partials row j at partials + j * row) into hist[j * nvec + v]
hipError_t launch_hist_finalize(const double *partials, size_t row, const VecDesc *vec, const int32_t *active, int nvec,
                                int k, double *hist, int32_t *bad, hipStream_t s);
// y (prec_dst) = x (prec_src), f = {y, x}
hipError_t launch_convert(int prec_dst, int prec_src, const BlasArgs &a, int block, hipStream_t s);

// pack.hip
hipError_t launch_pack_spinor(int prec, const PackArgs &a, int block, hipStream_t s);
hipError_t launch_unpack_spinor(int prec, const PackArgs &a, int block, hipStream_t s);
hipError_t launch_zero_canon(const PackArgs &a, int block, hipStream_t s);
hipError_t launch_pack_gauge(int prec, int recon, const double *U_canon, void *out, const SysDesc &d,
                             hipStream_t s);

// clover.hip: A = 1 + i kc sum_{m<n} s_mn F_mn from the canonical links, packed
// FP64, FP32 and FP16; then A^{-1} from the FP64 A
hipError_t launch_clover_build(const double *U_canon, const SysDesc &d, double kc, void *A64, void *A32, void *A16,
                               hipStream_t s);
hipError_t launch_clover_invert(const SysDesc &d, const void *A64, void *Ainv64, void *Ainv32, void *Ainv16,
                                hipStream_t s);
// mode 0: non-temporal copy; 1: cached copy; 2: cached read-only sum
hipError_t launch_copy_bw(int mode, const void *in, void *out, size_t bytes, hipStream_t s);

}  // namespace wl
