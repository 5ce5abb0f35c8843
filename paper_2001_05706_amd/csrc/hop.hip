// hop.hip -- the single-parity Wilson hopping kernel (the D-slash of Table 2)
// with a fused linear-combination epilogue and optional fused |out|^2.
//
// One thread per output site of one vector.  Per direction the neighbour
// spinor is spin-projected to two components (12 flop), both are multiplied
// by the link (2 x 66 flop) rebuilt from 12 reals when recon = 12, and the
// result is spin-reconstructed into the accumulator (24 flop): 1320 flop per
// site.  Each link is used once per hop and right-hand side; neighbour
// spinors are shared by up to 8 output sites through L2, which the XCD-aware
// block order keeps on one die.
#include <hip/hip_ext.h>

#include "wl_reduce.h"
#include "wl_kernels.h"

namespace wl {

// Launch variants the autotuner chooses from, with the block size:
//   fence: directions whose operands may be in flight together per wave
//   waves: occupancy target (waves per SIMD), which caps registers at 512/waves
//   nt:    non-temporal link loads or cached ones (cached win wherever a cache
//          line of links is shared: by the right-hand sides of a set, and by
//          neighbouring waves whose backward-link rows start mid line)
//   0: fence 2, 4 waves (FP64: 2), non-temporal links
//   1: fence 1, 5 waves (FP64: 3), non-temporal links
//   2: fence 1, 6 waves (FP64: 3), non-temporal links
//   3: fence 2, 4 waves (FP64: 2), cached links
//   4: fence 4, 4 waves, cached links -- twice the bytes in flight per wave
//   5: fence 4, 5 waves, cached links
//   6: as 3, but the waves of a block serve consecutive right-hand sides of one
//      system on the same 64 sites, so the links they share hit in the CU's L1
//      (multi-RHS sets; launched on the layouts of `ExecSet::layout(-G)`)
//   7: each thread serves two right-hand sides of one system at its site: the
//      neighbour index and each link (with its recon-12 row) are formed once
//      for both; one direction in flight, 3 waves (multi-RHS sets; pair layouts)
//   8: the waves of a block serve consecutive right-hand sides of one system on
//      the same 64 sites (as 6), and the block's 8 x 64 links are read, rebuilt
//      to 18 reals and stored in LDS once, together with the neighbour indices,
//      before any wave starts its hop: no right-hand side repeats a link load,
//      the recon-12 arithmetic or the site-coordinate arithmetic (FP32 and
//      half-precision storage; not with the clover epilogue)
//   9: pencil blocks (k_hop_pencil): the waves of a block take the same 64
//      positions of consecutive time slices and pass each other their time
//      neighbours through LDS; fence 2, non-temporal links
//  10: pencil blocks with cached links; fence 4 for FP16/BF16, 2 for FP32
//      (FP32 and half-precision storage, Wilson epilogue; lattices whose time
//      slices hold a multiple of 64 sites)
// Variants 4 and 5 exist for FP16/BF16 storage only (FP32 and FP64 operands of
// four directions do not fit the registers); for those they repeat variant 3.
template <int SP, int VAR> struct HopVar {
    static constexpr bool half = SP == P_F16 || SP == P_BF16;
    static constexpr int fence = VAR == 0 || VAR == 3 || VAR == 6 || VAR == 9
                                     ? 2
                                     : (VAR == 4 || VAR == 5 || VAR == 10 ? (half ? 4 : 2) : 1);
    static constexpr int waves = SP == P_F64 ? (VAR == 0 || VAR >= 3 ? 2 : 3)
                                             : (VAR == 7 ? 3 : VAR == 0 || VAR == 3 || VAR == 4 || VAR == 6 || VAR >= 9
                                                                   ? 4
                                                                   : VAR == 2 ? 6 : 5);
    static constexpr bool nt = VAR < 3 || VAR == 9;
    static constexpr bool rhs_waves = VAR == 6;
    static constexpr bool rhs_pairs = VAR == 7;
    // largest block: 1024 threads (16 waves on one CU, 4 per SIMD) where the
    // occupancy target already allows 4 waves per SIMD; 512 otherwise
    static constexpr int max_block = waves >= 4 && VAR < 6 ? 1024 : 512;
};
constexpr int kHopVariants = 11;

// The fields of the output parity a block computes: the launch's first slot,
// or for the second half of a twin launch the second one.  X and Xn point into
// the kernel's argument block, so that an index that varies at run time still
// reads them with scalar loads.
struct HopIO {
    int parity;
    const void *in;
    const float *in_norm;
    void *out;
    float *out_norm;
    const void *const *X;
    const float *const *Xn;
};

// Epilogue field X[j] at site cb, before its half-precision norm is applied.
// Each X field is read once per launch; for sets whose fields are large
// against the last-level cache the read is non-temporal, so that it does not
// push out the links that the solver's next hops re-read from that cache.
template <int SP>
__device__ __forceinline__ void load_x(const HopArgs &a, const HopIO &f, int j, size_t voff, const VecDesc &vd,
                                       const SysDesc &sd, int cb, typename SpinorFmt<SP>::real x[24],
                                       typename SpinorFmt<SP>::real *nx)
{
    using CH = typename SpinorFmt<SP>::chunk;
    const CH *base = (const CH *)f.X[j] + voff;
    const float *nrm = f.Xn[j] ? f.Xn[j] + vd.site_off : nullptr;
    if (a.stream)
        load_spinor_raw<SP, true>(base, nrm, sd.stride, cb, x, nx);
    else
        load_spinor_raw<SP, false>(base, nrm, sd.stride, cb, x, nx);
}

// Everything after the hopping sum at one output site of one vector: the
// linear-combination epilogue, the store, and the site's reduction values.
// acc holds H psi (FP16/BF16: already multiplied by the system's c).
template <int SP, bool CLOV>
__device__ __forceinline__ void hop_epilogue(const HopArgs &a, const HopIO &f, const VecDesc &vd, const SysDesc &sd,
                                             int cb, typename SpinorFmt<SP>::real acc[24], double rv[3])
{
    using T = typename SpinorFmt<SP>::real;
    using CH = typename SpinorFmt<SP>::chunk;
    constexpr int NC = SpinorFmt<SP>::nchunk;
    const size_t voff = (size_t)vd.site_off * NC;
    const double *cf = a.epi.coef + vd.sys * 5;
    constexpr bool HALF = SP == P_F16 || SP == P_BF16;
    // acc = c H psi from here on (half precision: c rode on the accumulation)
    if constexpr (!HALF) {
        const T c = (T)cf[4];
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] *= c;
    }

    // clover term of this system at the output site (FP16/BF16 launches read the FP16 copy)
    constexpr int CP = clover_prec<SP>();
    const bool clov = CLOV && a.epi.clov != 0 && sd.clov != nullptr;
    T o[24];
    if (a.epi.nx >= 1) {
        // operand values before their site norm; the norm joins the coefficient
        T x[24], n0 = 1;
        bool raw = true;
        if constexpr (CLOV) {
            if (clov && (a.epi.clov & EPI_CLOV_X0)) {
                load_spinor<SP>((const CH *)f.X[0] + voff, f.Xn[0] ? f.Xn[0] + vd.site_off : nullptr,
                                sd.stride, cb, x);
                clover_apply<CP>(clover_parity<CP>(sd.clov, f.parity, sd.stride), sd.stride, cb, x);
                n0 = 1;
                raw = false;
            }
        }
        if (raw) load_x<SP>(a, f, 0, voff, vd, sd, cb, x, &n0);
        const T s0 = (T)cf[0] * n0;
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] = fmadd(x[k], s0, acc[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] = acc[k];
    }
    if (a.epi.g5) {
#pragma unroll
        for (int k = 12; k < 24; ++k) o[k] = -o[k];
    }
    if constexpr (CLOV) {
        if (clov && (a.epi.clov & EPI_CLOV_INV))
            clover_apply<CP>(clover_parity<CP>(sd.clovinv, f.parity, sd.stride), sd.stride, cb, o);
    }
    for (int j = 1; j < a.epi.nx; ++j) {
        T x[24], nj;
        load_x<SP>(a, f, j, voff, vd, sd, cb, x, &nj);
        const T sj = (T)cf[j] * nj;
#pragma unroll
        for (int k = 0; k < 24; ++k) o[k] = fmadd(x[k], sj, o[k]);
    }
    store_spinor<SP, true>((CH *)f.out + voff, f.out_norm ? f.out_norm + vd.site_off : nullptr, sd.stride, cb, o);
    if (a.red.kind != RED_NONE) {
        if (a.red.mode == RM_NORM) {
            rv[0] = site_norm2(o);
        } else {
            // the X field was read above; this re-read hits in cache.  The
            // products are linear in x: its site norm scales the site sums.
            const int j = a.red.mode == RM_DOT_X1 ? 1 : 0;
            T x[24], nx;
            load_spinor_raw<SP>((const CH *)f.X[j] + voff, f.Xn[j] ? f.Xn[j] + vd.site_off : nullptr,
                                sd.stride, cb, x, &nx);
            if (a.red.mode == RM_DOT_X1) {
                site_cdot(x, o, rv[0], rv[1]);
            } else {
                site_cdot(o, x, rv[0], rv[1]);
                rv[2] = site_norm2(o);
            }
            rv[0] *= (double)nx;
            rv[1] *= (double)nx;
        }
    }
}

template <int SP>
__device__ __forceinline__ HopSite hop_input(const HopArgs &a, const HopIO &f, const VecDesc &vd, const SysDesc &sd)
{
    using CH = typename SpinorFmt<SP>::chunk;
    constexpr bool HALF = SP == P_F16 || SP == P_BF16;
    HopSite hs;
    hs.in = (const CH *)f.in + (size_t)vd.site_off * SpinorFmt<SP>::nchunk;
    hs.in_norm = f.in_norm ? f.in_norm + vd.site_off : nullptr;
    hs.stride = sd.stride;
    hs.gauge = sd.gauge;
    hs.gstride = sd.gstride;
    hs.scale = HALF ? (float)a.epi.coef[vd.sys * 5 + 4] : 1.0f;
    return hs;
}

template <int SP, int GP, int R, bool DAG, int VAR, bool CLOV>
__global__ __launch_bounds__((HopVar<SP, VAR>::max_block)) __attribute__((amdgpu_waves_per_eu(HopVar<SP, VAR>::waves)))
void k_hop(HopArgs a)
{
    using T = typename SpinorFmt<SP>::real;

    constexpr bool RW = HopVar<SP, VAR>::rhs_waves;
    constexpr bool PAIR = HopVar<SP, VAR>::rhs_pairs;
    const int lb = xcd_remap(blockIdx.x, a.nblocks);
    // a twin launch's second half computes the other output parity from the
    // second field slot (the selection is uniform over the block)
    const int half = a.nblocks >> 1;
    const bool second = a.twin && lb >= half;
    const HopIO f = second ? HopIO{1 - a.parity, a.in_b, a.in_norm_b, a.out_b, a.out_norm_b, a.X_b, a.Xn_b}
                           : HopIO{a.parity, a.in, a.in_norm, a.out, a.out_norm, a.epi.X, a.epi.Xn};
    const BlkMap bm = a.map[second ? lb - half : lb];
    int v = bm.v, cb;
    bool valid = true;
    if constexpr (RW) {
        // wave w serves vector bm.v + w (when it is a further rhs of the same system) on 64 sites
        // wave-uniform: keep the vector's descriptors in scalar registers
        const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
        v = bm.v + w;
        valid = v < a.nvec && a.vec[v].sys == a.vec[bm.v].sys && (!a.active || a.active[v]);
        cb = bm.lblk * 64 + ((int)threadIdx.x & 63);
    } else if constexpr (PAIR) {
        cb = bm.lblk * (int)blockDim.x + (int)threadIdx.x;
    } else {
        if (a.active && !a.active[a.one ? 0 : bm.v]) return;
        cb = bm.lblk * (int)blockDim.x + (int)threadIdx.x;
    }
    // (single-vector sets: the indices are known, so the descriptor loads do
    // not wait for the block map)
    const VecDesc vd = a.vec[a.one ? 0 : (valid ? v : bm.v)];
    const SysDesc sd = a.sys[a.one ? 0 : vd.sys];
    // the block's start stamp goes to memory at once, after the descriptor
    // loads are issued (held in registers across the body, or read before
    // them, it costs the FP16 kernel four registers and a spill)
    if (a.stamps && threadIdx.x == 0) a.stamps[2 * lb] = (unsigned long long)wall_clock64();

    if constexpr (PAIR) {
        // vectors bm.v and bm.v + 1 (when that is a further rhs of the same
        // system); an absent second vector is computed from the first and not stored
        const int v1 = bm.v + 1;
        const bool has1 = v1 < a.nvec && a.vec[v1].sys == vd.sys;
        const bool live0 = !a.active || a.active[bm.v];
        const bool live1 = has1 && (!a.active || a.active[v1]);
        if (!live0 && !live1) return;
        const VecDesc vd1 = a.vec[has1 ? v1 : bm.v];
        double rv0[3] = {0.0, 0.0, 0.0}, rv1[3] = {0.0, 0.0, 0.0};
        if (cb < sd.Vh) {
            const HopSite hs0 = hop_input<SP>(a, f, vd, sd), hs1 = hop_input<SP>(a, f, vd1, sd);
            T acc0[24], acc1[24];
            hop_site2<SP, GP, R, DAG, HopVar<SP, VAR>::nt>(sd, hs0, hs1, f.parity, cb, acc0, acc1);
            if (live0) hop_epilogue<SP, CLOV>(a, f, vd, sd, cb, acc0, rv0);
            if (live1) hop_epilogue<SP, CLOV>(a, f, vd1, sd, cb, acc1, rv1);
        }
        // live0 and live1 are uniform over the block
        if (a.red.kind != RED_NONE && live0) block_reduce_store_n(a.red, vd.pslot0, bm.lblk, rv0);
        if (a.red.kind != RED_NONE && live1) block_reduce_store_n(a.red, vd1.pslot0, bm.lblk, rv1);
    } else {
        double rv[3] = {0.0, 0.0, 0.0};
        if (valid && cb < sd.Vh) {
            const HopSite hs = hop_input<SP>(a, f, vd, sd);
            T acc[24];
            hop_site<SP, GP, R, DAG, HopVar<SP, VAR>::fence, HopVar<SP, VAR>::nt>(sd, hs, f.parity, cb, acc);
            hop_epilogue<SP, CLOV>(a, f, vd, sd, cb, acc, rv);
        }
        if constexpr (RW) {
            if (a.red.kind != RED_NONE && valid) wave_reduce_store_n(a.red, vd.pslot0, bm.lblk, rv);
        } else {
            if (a.red.kind != RED_NONE) block_reduce_store_n(a.red, vd.pslot0, bm.lblk, rv);
        }
    }
    if (a.stamps) {
        // the block's work ends when its last wave ends
        __syncthreads();
        if (threadIdx.x == 0) a.stamps[2 * lb + 1] = (unsigned long long)wall_clock64();
    }
}

// Variant 8.  LDS holds, per direction d = 2 mu + (backward), the rebuilt link
// of each of the block's 64 sites as 9 complex numbers ([d][element][site], so
// a wave's 64 lanes read 64 consecutive float2) and the neighbour's
// checkerboard index with the antiperiodic sign in bit 31: 38.9 KB per block.
constexpr int kLdsLinkBytes = 8 * 9 * 64 * (int)sizeof(float2) + 8 * 64 * (int)sizeof(int);

template <int GP, int R, int MU, int DIR>
__device__ __forceinline__ void stage_dir(const SysDesc &sd, const HopSite &hs, int parity, const Site &st, int cb,
                                          int lane, bool nt, float2 (*su)[64], int *sn)
{
    bool flip;
    const int ncb = neighbour<MU, DIR>(sd, st, cb, flip);
    cpx<float> u[3][3];
    if (nt)
        hop_link<GP, R, MU, DIR, true>(hs, parity, cb, ncb, u);
    else
        hop_link<GP, R, MU, DIR, false>(hs, parity, cb, ncb, u);
#pragma unroll
    for (int k = 0; k < 9; ++k) su[k][lane] = float2{u[k / 3][k % 3].re, u[k / 3][k % 3].im};
    sn[lane] = (int)((unsigned)ncb | (flip ? 0x80000000u : 0u));
}

template <int SP, int MU, int DIR, bool DAG>
__device__ __forceinline__ void lds_dir(const HopSite &hs, int lane, const float2 (*su)[64], const int *sn,
                                        float acc[24])
{
    constexpr int SG = (DIR > 0) == DAG ? +1 : -1;
    const int nn = sn[lane];
    cpx<float> h0[3], h1[3];
    const float f = project_neighbour<SP, MU, SG>(hs, nn & 0x7fffffff, nn < 0, h0, h1);
    cpx<float> u[3][3];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float2 w = su[k][lane];
        u[k / 3][k % 3] = cpx<float>{w.x, w.y};
    }
    hop_accumulate<SP, MU, DIR, SG>(u, h0, h1, f, acc);
}

template <int SP, int GP, int R, bool DAG>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) void k_hop_lds(HopArgs a)
{
    static_assert(SP != P_F64, "variant 8 stages FP32 links");
    __shared__ float2 s_u[8][9][64];
    __shared__ int s_n[8][64];
    static_assert(sizeof(s_u) + sizeof(s_n) == kLdsLinkBytes, "LDS layout of variant 8");
    const int lb = xcd_remap(blockIdx.x, a.nblocks);
    const int half = a.nblocks >> 1;
    const bool second = a.twin && lb >= half;
    const HopIO f = second ? HopIO{1 - a.parity, a.in_b, a.in_norm_b, a.out_b, a.out_norm_b, a.X_b, a.Xn_b}
                           : HopIO{a.parity, a.in, a.in_norm, a.out, a.out_norm, a.epi.X, a.epi.Xn};
    const BlkMap bm = a.map[second ? lb - half : lb];
    const int lane = (int)threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int nw = (int)blockDim.x >> 6;
    const int sys = a.vec[bm.v].sys;
    auto live = [&](int v) { return v < a.nvec && a.vec[v].sys == sys && (!a.active || a.active[v]); };
    // a block whose right-hand sides have all converged has nothing to do
    bool any = false;
    for (int k = 0; k < nw; ++k) any = any || live(bm.v + k);
    if (!any) return;
    const SysDesc sd = a.sys[sys];
    const int cb = bm.lblk * 64 + lane;
    if (a.stamps && threadIdx.x == 0) a.stamps[2 * lb] = (unsigned long long)wall_clock64();

    // stage: wave w rebuilds the links of directions w, w + nw, ... (all waves
    // take part, also those whose right-hand side is idle).  When the block
    // holds every right-hand side of its system, no other block reads these
    // links: they are loaded non-temporally.
    const bool nt = a.vec[bm.v].rhs == 0 && (bm.v + nw >= a.nvec || a.vec[bm.v + nw].sys != sys);
    if (cb < sd.Vh) {
        const Site st = cb_coords(sd, cb, f.parity);
        HopSite hl;
        hl.gauge = sd.gauge;
        hl.gstride = sd.gstride;
        for (int d = w; d < 8; d += nw) {
            switch (d) {
            case 0: stage_dir<GP, R, 0, +1>(sd, hl, f.parity, st, cb, lane, nt, s_u[0], s_n[0]); break;
            case 1: stage_dir<GP, R, 0, -1>(sd, hl, f.parity, st, cb, lane, nt, s_u[1], s_n[1]); break;
            case 2: stage_dir<GP, R, 1, +1>(sd, hl, f.parity, st, cb, lane, nt, s_u[2], s_n[2]); break;
            case 3: stage_dir<GP, R, 1, -1>(sd, hl, f.parity, st, cb, lane, nt, s_u[3], s_n[3]); break;
            case 4: stage_dir<GP, R, 2, +1>(sd, hl, f.parity, st, cb, lane, nt, s_u[4], s_n[4]); break;
            case 5: stage_dir<GP, R, 2, -1>(sd, hl, f.parity, st, cb, lane, nt, s_u[5], s_n[5]); break;
            case 6: stage_dir<GP, R, 3, +1>(sd, hl, f.parity, st, cb, lane, nt, s_u[6], s_n[6]); break;
            default: stage_dir<GP, R, 3, -1>(sd, hl, f.parity, st, cb, lane, nt, s_u[7], s_n[7]); break;
            }
        }
    }
    __syncthreads();

    const int v = bm.v + w;
    const bool valid = live(v);
    double rv[3] = {0.0, 0.0, 0.0};
    if (valid && cb < sd.Vh) {
        const VecDesc vd = a.vec[v];
        const HopSite hs = hop_input<SP>(a, f, vd, sd);
        float acc[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) acc[k] = 0.f;
        // two directions' operands in flight per wave, as variant 6
        lds_dir<SP, 0, +1, DAG>(hs, lane, s_u[0], s_n[0], acc);
        lds_dir<SP, 0, -1, DAG>(hs, lane, s_u[1], s_n[1], acc);
        sched_fence(acc);
        lds_dir<SP, 1, +1, DAG>(hs, lane, s_u[2], s_n[2], acc);
        lds_dir<SP, 1, -1, DAG>(hs, lane, s_u[3], s_n[3], acc);
        sched_fence(acc);
        lds_dir<SP, 2, +1, DAG>(hs, lane, s_u[4], s_n[4], acc);
        lds_dir<SP, 2, -1, DAG>(hs, lane, s_u[5], s_n[5], acc);
        sched_fence(acc);
        lds_dir<SP, 3, +1, DAG>(hs, lane, s_u[6], s_n[6], acc);
        lds_dir<SP, 3, -1, DAG>(hs, lane, s_u[7], s_n[7], acc);
        sched_fence(acc);
        hop_epilogue<SP, false>(a, f, vd, sd, cb, acc, rv);
    }
    if (a.red.kind != RED_NONE && valid) wave_reduce_store_n(a.red, a.vec[v].pslot0, bm.lblk, rv);
    if (a.stamps) {
        __syncthreads();
        if (threadIdx.x == 0) a.stamps[2 * lb + 1] = (unsigned long long)wall_clock64();
    }
}

// Variants 9 and 10: pencil blocks.  The nw = block / 64 waves of a block
// take the same 64 positions of nw consecutive time slices of one vector
// (wave j: slice t0 + j; the set's slices hold a multiple of 64 sites and nw
// divides the time extent).  In the checkerboard index the time neighbours of
// output site cb are the input sites cb +- (sites per slice), at the same
// position: the input row at wave j's own sites is the forward time
// neighbour of wave j - 1 and the backward one of wave j + 1.  Each wave puts
// that row into LDS once; inside the block the time directions read it there,
// and only the outer slices fetch a time row from memory.  (The stand-alone
// hop fetches every input spinor about twice, and the second fetch is the
// time rows'.)  LDS holds per wave the row's raw chunks, [chunk][lane], and
// for FP16/BF16 its norms.  Every direction runs the per-site arithmetic of
// hop_site in its order, so the result equals the other variants' bit for bit.
template <int SP> struct PencilRow {
    using CH = typename SpinorFmt<SP>::chunk;
    static constexpr int NC = SpinorFmt<SP>::nchunk;
    static constexpr bool HALF = SP == P_F16 || SP == P_BF16;
    static constexpr int chunk_bytes = NC * 64 * (int)sizeof(CH);
    static constexpr int bytes = chunk_bytes + (HALF ? 64 * (int)sizeof(float) : 0);
};

// the time direction DIR of output site cb from the neighbour row in LDS
// (interior slices of the block: no wrap, no boundary sign)
template <int SP, int GP, int R, int DIR, bool DAG, bool NT>
__device__ __forceinline__ void pencil_t(const HopSite &hs, int parity, int cb, int ncb, const unsigned char *row,
                                         int lane, float acc[24])
{
    using P = PencilRow<SP>;
    constexpr int SG = (DIR > 0) == DAG ? +1 : -1;
    const typename P::CH *src = reinterpret_cast<const typename P::CH *>(row);
    cpx<float> h0[3], h1[3];
    float f;
    if constexpr (P::HALF) {
        uint32_t q[12];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint4 w = src[c * 64 + lane];
            q[4 * c] = w.x;
            q[4 * c + 1] = w.y;
            q[4 * c + 2] = w.z;
            q[4 * c + 3] = w.w;
        }
        const float nrm = reinterpret_cast<const float *>(row + P::chunk_bytes)[lane];
        project_half<SP, 3, SG>(q, h0, h1);
        f = nrm * hs.scale;
    } else {
        float v[24];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const float4 w = src[c * 64 + lane];
            v[4 * c] = w.x;
            v[4 * c + 1] = w.y;
            v[4 * c + 2] = w.z;
            v[4 * c + 3] = w.w;
        }
        project<3, SG>(v, h0, h1);
        f = 1.f;
    }
    cpx<float> u[3][3];
    hop_link<GP, R, 3, DIR, NT>(hs, parity, cb, ncb, u);
    hop_accumulate<SP, 3, DIR, SG>(u, h0, h1, f, acc);
}

template <int SP, int GP, int R, bool DAG, int VAR>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(HopVar<SP, VAR>::waves)))
void k_hop_pencil(HopArgs a)
{
    static_assert(SP != P_F64, "pencil rows hold FP32 or half-precision spinors");
    using P = PencilRow<SP>;
    using CH = typename P::CH;
    constexpr int FENCE = HopVar<SP, VAR>::fence;
    constexpr bool NT = HopVar<SP, VAR>::nt;
    extern __shared__ uint4 s_pencil[];
    unsigned char *rows = reinterpret_cast<unsigned char *>(s_pencil);

    const int lb = xcd_remap(blockIdx.x, a.nblocks);
    const BlkMap bm = a.map[lb];
    if (a.active && !a.active[a.one ? 0 : bm.v]) return;  // uniform over the block
    const VecDesc vd = a.vec[a.one ? 0 : bm.v];
    const SysDesc sd = a.sys[a.one ? 0 : vd.sys];
    if (a.stamps && threadIdx.x == 0) a.stamps[2 * lb] = (unsigned long long)wall_clock64();
    const HopIO f{a.parity, a.in, a.in_norm, a.out, a.out_norm, a.epi.X, a.epi.Xn};
    const int lane = (int)threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int nw = (int)blockDim.x >> 6;
    const int slice = sd.Lxh * sd.L[1] * sd.L[2], nch = slice >> 6;
    const int pz = bm.lblk / nch;
    const int cb = (pz * nw + w) * slice + (bm.lblk - pz * nch) * 64 + lane;
    const HopSite hs = hop_input<SP>(a, f, vd, sd);

    // this wave's row: the input site at the thread's own index
    unsigned char *own = rows + w * P::bytes;
#pragma unroll
    for (int c = 0; c < P::NC; ++c)
        reinterpret_cast<CH *>(own)[c * 64 + lane] = ld_field<false>(row_elem<CH>(hs.in, c, hs.stride, cb));
    if constexpr (P::HALF)
        reinterpret_cast<float *>(own + P::chunk_bytes)[lane] = ld_field<false>(row_elem<float>(hs.in_norm, 0, 0, cb));

    float acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0.f;
    const Site st = cb_coords(sd, cb, f.parity);
    hop_dir<SP, GP, R, 0, +1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    hop_dir<SP, GP, R, 0, -1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    if constexpr (FENCE <= 2) sched_fence(acc);
    hop_dir<SP, GP, R, 1, +1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    hop_dir<SP, GP, R, 1, -1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    sched_fence(acc);
    __syncthreads();  // every wave's row is in LDS
    hop_dir<SP, GP, R, 2, +1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    hop_dir<SP, GP, R, 2, -1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    if constexpr (FENCE <= 2) sched_fence(acc);
    if (w + 1 < nw)
        pencil_t<SP, GP, R, +1, DAG, NT>(hs, f.parity, cb, cb + slice, rows + (w + 1) * P::bytes, lane, acc);
    else
        hop_dir<SP, GP, R, 3, +1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    if (w > 0)
        pencil_t<SP, GP, R, -1, DAG, NT>(hs, f.parity, cb, cb - slice, rows + (w - 1) * P::bytes, lane, acc);
    else
        hop_dir<SP, GP, R, 3, -1, DAG, NT>(sd, hs, f.parity, st, cb, acc);
    sched_fence(acc);

    double rv[3] = {0.0, 0.0, 0.0};
    hop_epilogue<SP, false>(a, f, vd, sd, cb, acc, rv);
    if (a.red.kind != RED_NONE) block_reduce_store_n(a.red, vd.pslot0, bm.lblk, rv);
    if (a.stamps) {
        __syncthreads();
        if (threadIdx.x == 0) a.stamps[2 * lb + 1] = (unsigned long long)wall_clock64();
    }
}

// With events, the dispatch itself records them at the kernel's start and end
// (the kernel-timing form of the launch), so the measured interval is the
// kernel alone.
template <class K>
static void dispatch(K kernel, const HopArgs &a, int block, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                     unsigned lds = 0)
{
    if (e0)
        hipExtLaunchKernelGGL(kernel, dim3(a.nblocks), dim3(block), lds, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(kernel, dim3(a.nblocks), dim3(block), lds, s, a);
}

template <int SP, int GP, int R, int VAR>
static hipError_t launch_hop_v(bool dag, bool clov, const HopArgs &a, int block, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1)
{
    // the clover epilogue is a separate instantiation: it needs registers the Wilson kernels do not
    if (dag && clov)
        dispatch(k_hop<SP, GP, R, true, VAR, true>, a, block, s, e0, e1);
    else if (dag)
        dispatch(k_hop<SP, GP, R, true, VAR, false>, a, block, s, e0, e1);
    else if (clov)
        dispatch(k_hop<SP, GP, R, false, VAR, true>, a, block, s, e0, e1);
    else
        dispatch(k_hop<SP, GP, R, false, VAR, false>, a, block, s, e0, e1);
    return hipGetLastError();
}

template <int SP, int GP, int R>
static hipError_t launch_hop_t(int var, bool dag, bool clov, const HopArgs &a, int block, hipStream_t s,
                               hipEvent_t e0, hipEvent_t e1)
{
    switch (var) {
    case 0: return launch_hop_v<SP, GP, R, 0>(dag, clov, a, block, s, e0, e1);
    case 1: return launch_hop_v<SP, GP, R, 1>(dag, clov, a, block, s, e0, e1);
    case 2: return launch_hop_v<SP, GP, R, 2>(dag, clov, a, block, s, e0, e1);
    case 3: return launch_hop_v<SP, GP, R, 3>(dag, clov, a, block, s, e0, e1);
    case 4: return launch_hop_v<SP, GP, R, 4>(dag, clov, a, block, s, e0, e1);
    case 5: return launch_hop_v<SP, GP, R, 5>(dag, clov, a, block, s, e0, e1);
    case 6: return launch_hop_v<SP, GP, R, 6>(dag, clov, a, block, s, e0, e1);
    case 7: return launch_hop_v<SP, GP, R, 7>(dag, clov, a, block, s, e0, e1);
    case 8:
        if constexpr (SP != P_F64) {
            if (clov || block % 64 != 0 || block > 1024) return hipErrorInvalidValue;
            if (dag)
                dispatch(k_hop_lds<SP, GP, R, true>, a, block, s, e0, e1);
            else
                dispatch(k_hop_lds<SP, GP, R, false>, a, block, s, e0, e1);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    case 9:
    case 10:
        if constexpr (SP != P_F64) {
            // 2 to 8 slices per block, one vector per block, no twin launch
            if (clov || a.twin || block % 64 != 0 || block < 128 || block > 512) return hipErrorInvalidValue;
            const unsigned lds = (unsigned)(block / 64 * PencilRow<SP>::bytes);
            if (var == 9)
                dispatch(dag ? k_hop_pencil<SP, GP, R, true, 9> : k_hop_pencil<SP, GP, R, false, 9>, a, block, s, e0,
                         e1, lds);
            else
                dispatch(dag ? k_hop_pencil<SP, GP, R, true, 10> : k_hop_pencil<SP, GP, R, false, 10>, a, block, s,
                         e0, e1, lds);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

// FP64 runs variants 0-7 (variants 8-10 stage FP32 or half-precision data in LDS)
int hop_variants(int prec) { return prec == P_F64 ? 8 : kHopVariants; }

hipError_t launch_hop(int prec, int recon, bool dag, bool clov, int var, const HopArgs &a, int block, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1)
{
    if (prec == P_F64 && recon == 18) return launch_hop_t<P_F64, P_F64, 18>(var, dag, clov, a, block, s, e0, e1);
    if (prec == P_F64 && recon == 12) return launch_hop_t<P_F64, P_F64, 12>(var, dag, clov, a, block, s, e0, e1);
    if (prec == P_F32 && recon == 18) return launch_hop_t<P_F32, P_F32, 18>(var, dag, clov, a, block, s, e0, e1);
    if (prec == P_F32 && recon == 12) return launch_hop_t<P_F32, P_F32, 12>(var, dag, clov, a, block, s, e0, e1);
    if (prec == P_F16 && recon == 12) return launch_hop_t<P_F16, P_F16, 12>(var, dag, clov, a, block, s, e0, e1);
    if (prec == P_BF16 && recon == 12) return launch_hop_t<P_BF16, P_BF16, 12>(var, dag, clov, a, block, s, e0, e1);
    return hipErrorInvalidValue;
}

}  // namespace wl
