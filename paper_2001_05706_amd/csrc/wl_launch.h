// wl_launch.h -- launch descriptors shared by the host driver and the kernels.
//
// A launch covers a set of "vectors" (one right-hand side of one system on one
// parity) that may belong to systems of different lattice sizes.  The
// per-system descriptors (SysDesc), per-vector descriptors (VecDesc) and the
// block map live in device memory and are read by reference, so kernel
// arguments stay small whatever the batch size.
#pragma once

#include "wl_core.h"

namespace wl {

struct VecDesc {
    int32_t sys;       // system index
    int32_t rhs;       // right-hand side within the system
    int32_t site_off;  // offset of this vector, in sites, inside every field of the set
    int32_t nblk;      // blocks of this vector in the current block size
    int32_t pslot0;    // first partial-sum slot
    int32_t pad_;
};

// Logical block -> (vector, block within the vector).  Logical order is
// (system, site block, rhs), so right-hand sides sharing links are adjacent
// and land on the same XCD after the XCD remap.
struct BlkMap {
    int32_t v;
    int32_t lblk;
};

// Map the hardware block id to a logical block so that the 8 XCDs (which
// receive hardware blocks round-robin) each own one contiguous range of
// logical blocks: neighbouring sites then share one L2.
WL_HD int xcd_remap(int h, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int k = h & 7, i = h >> 3;
    return k * q + (k < r ? k : r) + i;
}

// Per-vector scalar slots of a set: scalar `slot` of vector v lives at
// sc[slot * nvec + v].  Complex scalars use two slots (re, im).
enum ScSlot {
    SC_ALPHA = 0, SC_BETA, SC_GAM, SC_QQ, SC_RR, SC_ETA, SC_TMP,
    SC_RHO_RE, SC_RHO_IM,      // BiCGStab rho = <rhat, r>
    SC_RHOP_RE, SC_RHOP_IM,    // rho of the previous iteration
    SC_AL_RE, SC_AL_IM,        // complex alpha
    SC_OM_RE, SC_OM_IM,        // complex omega
    SC_COUNT
};

// Reduction of per-site values (1 to 3 FP64 numbers per vector: block
// partials, then a fixed-order finishing pass), and the finishing step.
enum RedKind {
    RED_NONE = 0,
    RED_STORE = 1,        // dst[v] = s0
    RED_ALPHA = 2,        // alpha = gam / s0           (s0 = |q|^2)
    RED_BETA = 3,         // beta = s0 / gam; gam = s0
    RED_GAMMA = 4,        // gam = s0
    RED_ACCUM = 5,        // dst[v] += s0
    RED_CDOT_RHO = 6,     // rho = s0 + i s1
    RED_BICG_ALPHA = 7,   // alpha = rho / (s0 + i s1); rho_prev = rho
    RED_BICG_OMEGA = 8,   // omega = (s0 + i s1) / s2
    RED_BICG_RHO = 9,     // rho = s0 + i s1; dst[v] = s2
    RED_BICG_INIT = 10,   // rho = rho_prev = s0 + i s1; alpha = omega = 1
    RED_CSTORE = 11,      // dst[2v] = s0, dst[2v+1] = s1
    RED_CACCUM = 12,      // dst[2v] += s0, dst[2v+1] += s1
};

// What the hop epilogue reduces (RedSpec::mode)
enum RedMode {
    RM_NORM = 0,    // |out|^2                             (1 value)
    RM_DOT_X1 = 1,  // <X1, out>                            (2 values)
    RM_OUT_X0 = 2,  // <out, X0>, |out|^2                   (3 values)
};

struct RedSpec {
    int32_t kind;
    int32_t nv;          // values per site (1..3)
    int32_t mode;        // RedMode for hop epilogues
    int32_t nvec;        // vectors of the set (scalar-slot stride)
    double *partials;    // per (vector, block) partial sums, nv values each
    double *sc;          // scalar slots (ScSlot)
    double *dst;         // RED_STORE / RED_ACCUM / RED_BICG_RHO target, indexed by vector
    int32_t *bad;        // per-vector non-finite flag (bit 0)
    int32_t defer;       // 1: leave the partials for a later finishing pass (no finishing launch)
    int32_t pad_;
};

// Linear combination applied to the hopping term at the output site:
//   out = Ci G5?( a0 C0 X0 + c hop ) + a1 X1 + a2 X2 + a3 X3
// with coefficients per system in device memory: coef[sys * 5 + {0..3: a0..a3, 4: c}].
// The X fields share the output's precision and parity.  For a system with a
// clover term, C0 = A (clov bit 0) and Ci = A^{-1} (clov bit 1) at the output
// site; otherwise both are 1.
enum { EPI_CLOV_X0 = 1, EPI_CLOV_INV = 2 };
struct EpiSpec {
    int32_t nx;          // number of X fields used (0..4)
    int32_t g5;          // apply gamma_5 to (a0 X0 + c hop)
    int32_t clov;        // EPI_CLOV_* bits
    int32_t pad_;
    const double *coef;
    const void *X[4];
    const float *Xn[4];  // norms for FP16/BF16
};

// Everything a hop launch needs besides the system and vector tables.
struct HopArgs {
    const SysDesc *sys;
    const VecDesc *vec;
    const BlkMap *map;
    const int32_t *active;  // per-vector mask (NULL: all active)
    int32_t nblocks;
    int32_t parity;         // output parity
    int32_t nvec;           // vectors of the set
    int32_t stream;         // epilogue X fields read non-temporally
    const void *in;         // field bases (all vectors of the set)
    const float *in_norm;
    void *out;
    float *out_norm;
    EpiSpec epi;
    RedSpec red;
    // kernel timing (null: off): each block stores its first and last steady-clock
    // reading at stamps[2 * logical block + {0, 1}]
    unsigned long long *stamps;
    // one == 1: the set is a single vector (vector 0 of system 0), so a block
    // loads its descriptors without waiting for the block map
    int32_t one;
    // twin == 1: the launch covers both output parities: logical blocks
    // [nblocks/2, nblocks) repeat the block map for output parity 1 - parity,
    // reading the fields of the second slot below (no reduction)
    int32_t twin;
    const void *in_b;
    const float *in_norm_b;
    void *out_b;
    float *out_norm_b;
    const void *X_b[4];
    const float *Xn_b[4];
};

}  // namespace wl
