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

// Reduction of a per-site scalar to one FP64 number per vector (block partials,
// then a fixed-order finishing pass), and the finishing step applied to it.
enum RedKind {
    RED_NONE = 0,
    RED_STORE = 1,   // dst[v] = sum
    RED_ALPHA = 2,   // alpha[v] = gam[v] / sum        (sum = |q|^2)
    RED_BETA = 3,    // beta[v] = sum / gam[v]; gam[v] = sum
    RED_GAMMA = 4,   // gam[v] = sum
    RED_ACCUM = 5,   // dst[v] += sum
};

struct RedSpec {
    int32_t kind;
    int32_t pad_;
    double *partials;    // per (vector, block) partial sums
    uint32_t *counters;  // reserved
    double *dst;         // RED_STORE target, indexed by vector
    double *gam;
    double *alpha;
    double *beta;
    int32_t *bad;        // per-vector non-finite flag (bit 0)
};

// Linear combination applied to the hopping term at the output site:
//   out = G5?( a0 X0 + c hop ) + a1 X1 + a2 X2 + a3 X3
// with coefficients per system in device memory: coef[sys * 5 + {0..3: a0..a3, 4: c}].
// The X fields share the output's precision and parity.
struct EpiSpec {
    int32_t nx;          // number of X fields used (0..4)
    int32_t g5;          // apply gamma_5 to (a0 X0 + c hop)
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
    const void *in;         // field bases (all vectors of the set)
    const float *in_norm;
    void *out;
    float *out_norm;
    EpiSpec epi;
    RedSpec red;
};

}  // namespace wl
