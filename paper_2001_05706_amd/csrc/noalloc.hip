// noalloc.hip -- the D-slash entry point that allocates nothing.
//
// wilson_dslash_noalloc computes what wilson_dslash computes, with the same
// kernels, but every buffer beyond the caller's input and output fields lives
// in one file-scope device array `scratch` of kNoAllocBytes: the descriptor
// tables, the coefficient row, the links packed from the handle's canonical
// copy, and the packed input and output fields.  No hipMalloc, hipFree or
// memset is issued, so the call can be made where allocating is not allowed
// (for instance while a stream is being captured into a graph).
//
// The array's host-side name is only a stand-in for the symbol: its device
// address is fetched once per device with hipGetSymbolAddress and that
// address is what the kernels receive.  Every call on one device shares the
// array: calls that overlap on one device (several streams, several host
// threads) race, and the caller must order them.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "wl_host.h"

namespace wl {

constexpr size_t kNoAllocBytes = (size_t)WL_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocDevices = 64;
constexpr int kNoAllocBlock = 256;  // sites per block: pack, hop and unpack share one block map
constexpr int kNoAllocVariant = 3;  // hop launch variant: two directions in flight, cached link loads

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kNoAllocDevices] = {};

// The device address of `scratch` on the current device (looked up once per device).
static wl_status scratch_address(void **out)
{
    int dev = 0;
    WL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) return set_error(WL_ERR_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(WL_ERR_HIP, "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return WL_OK;
}

// Descriptor tables of one system with nrhs vectors in blocks of kNoAllocBlock
// sites, ordered (site block, rhs) so that the right-hand sides of a block's
// sites run next to each other; and the epilogue's coefficient row.
__global__ void k_noalloc_setup(SysDesc sd, int nrhs, int nb, double c0, double c4, SysDesc *sys, VecDesc *vec,
                                BlkMap *map, double *coef)
{
    const int n = nb * nrhs;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        map[i] = BlkMap{i % nrhs, i / nrhs};
        if (i < nrhs) vec[i] = VecDesc{0, i, i * sd.stride, nb, i * nb, 0};
        if (i == 0) {
            *sys = sd;
            coef[0] = c0;
            coef[1] = coef[2] = coef[3] = 0.0;
            coef[4] = c4;
        }
    }
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace wl

using namespace wl;

namespace wl {
wl_status check_gauge(wl_gauge U);
wl_status check_field(const void *p, wl_gauge U, int nrhs, const char *what);
}  // namespace wl

extern "C" wl_status wilson_dslash_noalloc(wl_gauge U, const double *in, double *out, int32_t nrhs, double kappa,
                                           int32_t parity, int32_t dagger, wl_prec prec, int32_t recon, void *stream)
{
    clear_error();
    WL_TRY(check_gauge(U));
    if (nrhs < 1) return set_error(WL_ERR_ARG, "nrhs = %d must be >= 1", nrhs);
    if (parity < -1 || parity > 1) return set_error(WL_ERR_ARG, "parity must be -1, 0 or 1");
    if (dagger != 0 && dagger != 1) return set_error(WL_ERR_ARG, "dagger must be 0 or 1");
    if (!std::isfinite(kappa)) return set_error(WL_ERR_ARG, "kappa must be finite");
    if (!prec_recon_ok(prec, recon)) return set_error(WL_ERR_PREC, "unsupported precision %d / recon %d", prec, recon);
    WL_TRY(check_field(in, U, nrhs, "in"));
    WL_TRY(check_field(out, U, nrhs, "out"));
    const size_t cbytes = (size_t)nrhs * 2 * U->geom.Vh * 24 * sizeof(double);
    if ((const char *)in < (const char *)out + cbytes && (const char *)out < (const char *)in + cbytes)
        return set_error(WL_ERR_ARG, "in and out overlap");
    int dev = 0;
    WL_HIP(hipGetDevice(&dev));
    if (dev != U->device) return set_error(WL_ERR_ARG, "the handle lives on device %d, the current device is %d",
                                           U->device, dev);

    // scratch layout: coefficient row, system, vectors, block map, links, then the
    // packed fields (inputs then outputs, one per parity used), each 256-byte aligned
    const SysDesc &g = U->geom;
    const int nb = (g.Vh + kNoAllocBlock - 1) / kNoAllocBlock;
    const size_t nblocks = (size_t)nb * nrhs;
    const size_t lbytes = (size_t)2 * 4 * g.gstride * link_bytes(prec, recon);  // both parities, 4 directions
    const size_t fbytes = (size_t)nrhs * g.stride * nchunks(prec) * chunk_bytes(prec);
    const bool half = prec == P_F16 || prec == P_BF16;
    const size_t nbytes = half ? (size_t)nrhs * g.stride * sizeof(float) : 0;
    const int nfield = parity < 0 ? 2 : 1;  // parities of input (and of output)
    size_t off = 0;
    const size_t o_coef = off;
    off += align256(5 * sizeof(double));
    const size_t o_sys = off;
    off += align256(sizeof(SysDesc));
    const size_t o_vec = off;
    off += align256((size_t)nrhs * sizeof(VecDesc));
    const size_t o_map = off;
    off += align256(nblocks * sizeof(BlkMap));
    const size_t o_links = off;
    off += align256(lbytes);
    size_t o_f[2][2], o_n[2][2];  // [input / output][slot]
    for (int io = 0; io < 2; ++io)
        for (int k = 0; k < nfield; ++k) {
            o_f[io][k] = off;
            off += align256(fbytes);
            o_n[io][k] = off;
            off += align256(nbytes);
        }
    if (off > kNoAllocBytes)
        return set_error(WL_ERR_ARG,
                         "this lattice and nrhs need %zu bytes of scratch; wilson_dslash_noalloc holds at most %zu "
                         "(use wilson_dslash)",
                         off, kNoAllocBytes);

    void *base = nullptr;
    WL_TRY(scratch_address(&base));
    char *b = (char *)base;
    double *coef = (double *)(b + o_coef);
    SysDesc *sys = (SysDesc *)(b + o_sys);
    VecDesc *vec = (VecDesc *)(b + o_vec);
    BlkMap *map = (BlkMap *)(b + o_map);
    void *links = b + o_links;
    auto field = [&](int io, int k) {
        Field f;
        f.p = b + o_f[io][k];
        f.n = half ? (float *)(b + o_n[io][k]) : nullptr;
        f.prec = prec;
        return f;
    };

    hipStream_t s = (hipStream_t)stream;
    SysDesc sd = g;
    sd.gauge = links;
    sd.clov = sd.clovinv = nullptr;
    // parity 0/1: out_p = hop(in_{1-p}); parity -1: out = in - kappa hop(in)
    const double c0 = parity < 0 ? 1.0 : 0.0, c4 = parity < 0 ? -kappa : 1.0;
    const int sblocks = (int)std::min<size_t>((nblocks + 255) / 256, 1024);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(sblocks), dim3(256), 0, s, sd, (int)nrhs, nb, c0, c4, sys, vec, map,
                       coef);
    WL_HIP(hipGetLastError());
    WL_HIP(launch_pack_gauge(prec, recon, U->U, links, g, s));

    PackArgs pa{};
    pa.sys = sys;
    pa.vec = vec;
    pa.map = map;
    pa.nblocks = (int)nblocks;
    pa.canon[0] = in;
    HopArgs ha{};
    ha.sys = sys;
    ha.vec = vec;
    ha.map = map;
    ha.active = nullptr;
    ha.nblocks = (int)nblocks;
    ha.nvec = nrhs;
    ha.epi.coef = coef;
    ha.red = RedSpec{};
    ha.red.kind = RED_NONE;
    ha.red.nv = 1;
    ha.one = nrhs == 1;
    // input slot k holds parity (parity < 0 ? k : 1 - parity); output slot k parity (parity < 0 ? k : parity)
    for (int k = 0; k < nfield; ++k) {
        const Field fi = field(0, k);
        pa.parity = parity < 0 ? k : 1 - parity;
        pa.f = fi.p;
        pa.fn = fi.n;
        WL_HIP(launch_pack_spinor(prec, pa, kNoAllocBlock, s));
    }
    for (int k = 0; k < nfield; ++k) {
        const int op = parity < 0 ? k : parity;  // output parity
        const Field fo = field(1, k), fin = field(0, parity < 0 ? 1 - k : 0);
        ha.parity = op;
        ha.in = fin.p;
        ha.in_norm = fin.n;
        ha.out = fo.p;
        ha.out_norm = fo.n;
        if (parity < 0) {
            const Field x0 = field(0, k);
            ha.epi.nx = 1;
            ha.epi.X[0] = x0.p;
            ha.epi.Xn[0] = x0.n;
        }
        WL_HIP(launch_hop(prec, recon, dagger != 0, false, kNoAllocVariant, ha, kNoAllocBlock, s));
    }
    pa.canon[0] = out;
    for (int k = 0; k < nfield; ++k) {
        const Field fo = field(1, k);
        pa.parity = parity < 0 ? k : parity;
        pa.f = fo.p;
        pa.fn = fo.n;
        WL_HIP(launch_unpack_spinor(prec, pa, kNoAllocBlock, s));
    }
    if (parity >= 0) {
        pa.parity = 1 - parity;
        pa.f = nullptr;
        pa.fn = nullptr;
        WL_HIP(launch_zero_canon(pa, kNoAllocBlock, s));
    }
    return WL_OK;
}
