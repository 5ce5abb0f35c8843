// hop_emu.hip -- host build of the GPU hop's per-site code, for CPU tests.
//
// The D-slash kernel's per-site arithmetic (packed loads with FP16/BF16
// dequantisation, recon-12 rebuild, spin projection, SU(3) products,
// reconstruction) is __host__ __device__; this file runs that same code on the
// host over every output site so that its indexing and algebra can be checked
// against the oracle without a GPU.  Test infrastructure only.
#include <vector>

#include "../paper_2001_05706_amd/csrc/wl_launch.h"

using namespace wl;

template <int P, int R, bool DAG>
static void emu(const int32_t *L, int tap, const double *U, const double *in, double *out, int parity)
{
    using SF = SpinorFmt<P>;
    using T = typename SF::real;
    SysDesc d{};
    for (int m = 0; m < 4; ++m) d.L[m] = L[m];
    d.Lxh = L[0] / 2;
    d.Vh = L[0] * L[1] * L[2] * L[3] / 2;
    d.stride = (d.Vh + 63) / 64 * 64 + 64;  // padding differs from the library on purpose
    d.gstride = d.stride + 64;
    d.tap = tap;
    set_divisors(d);
    constexpr int NCH = LinkFmt<P, R>::nchunk;
    using LCH = typename LinkFmt<P, R>::chunk;
    std::vector<LCH> links((size_t)8 * NCH * d.gstride);
    std::vector<typename SF::chunk> sp((size_t)SF::nchunk * d.stride);
    std::vector<float> nrm(d.stride);
    for (int par = 0; par < 2; ++par)
        for (int cb = 0; cb < d.Vh; ++cb) {
            Site s = cb_coords(d, cb, par);
            size_t lex = s.x + (size_t)L[0] * (s.y + (size_t)L[1] * (s.z + (size_t)L[2] * s.t));
            for (int mu = 0; mu < 4; ++mu)
                store_link<P, R>(links.data() + (size_t)((par * 4 + mu) * NCH) * d.gstride, d.gstride, cb,
                                 U + (lex * 4 + mu) * 18);
            if (par == 1 - parity) {
                T v[24];
                for (int k = 0; k < 24; ++k) v[k] = (T)in[lex * 24 + k];
                store_spinor<P>(sp.data(), nrm.data(), d.stride, cb, v);
            }
        }
    d.gauge = links.data();
    HopSite hs;
    hs.in = sp.data();
    hs.in_norm = nrm.data();
    hs.stride = d.stride;
    hs.gauge = links.data();
    hs.gstride = d.gstride;
    for (int cb = 0; cb < d.Vh; ++cb) {
        T acc[24];
        hop_site<P, P, R, DAG>(d, hs, parity, cb, acc);
        Site s = cb_coords(d, cb, parity);
        size_t lex = s.x + (size_t)L[0] * (s.y + (size_t)L[1] * (s.z + (size_t)L[2] * s.t));
        for (int k = 0; k < 24; ++k) out[lex * 24 + k] = (double)acc[k];
    }
}

template <int P, int R>
static void emu_d(int dag, const int32_t *L, int tap, const double *U, const double *in, double *out, int parity)
{
    if (dag)
        emu<P, R, true>(L, tap, U, in, out, parity);
    else
        emu<P, R, false>(L, tap, U, in, out, parity);
}

// out (canonical, V x 24 doubles) receives H in on the sites of `parity`
extern "C" int emu_hop(int prec, int recon, int dag, const int32_t *L, int tap, const double *U, const double *in,
                       double *out, int parity)
{
    if (prec == P_F64 && recon == 18) emu_d<P_F64, 18>(dag, L, tap, U, in, out, parity);
    else if (prec == P_F64 && recon == 12) emu_d<P_F64, 12>(dag, L, tap, U, in, out, parity);
    else if (prec == P_F32 && recon == 18) emu_d<P_F32, 18>(dag, L, tap, U, in, out, parity);
    else if (prec == P_F32 && recon == 12) emu_d<P_F32, 12>(dag, L, tap, U, in, out, parity);
    else if (prec == P_F16 && recon == 12) emu_d<P_F16, 12>(dag, L, tap, U, in, out, parity);
    else if (prec == P_BF16 && recon == 12) emu_d<P_BF16, 12>(dag, L, tap, U, in, out, parity);
    else return 1;
    return 0;
}

// xcd_remap over a whole grid, for the bijectivity test
extern "C" void emu_xcd_remap(int nb, int32_t *out)
{
    for (int h = 0; h < nb; ++h) out[h] = xcd_remap(h, nb);
}

// Checks idiv (the floating-point quotient of the coordinate code) against the
// integer quotient for every divisor 1..dmax, at the multiples k d - 1, k d,
// k d + 1 of the first and last 300 quotients below 2^26 and of 200 more spread
// between them.  Returns the number of disagreements.
extern "C" long emu_idiv_check(int dmax)
{
    long bad = 0;
    const int64_t nmax = (int64_t)1 << 26;
    for (int d = 1; d <= dmax; ++d) {
        const double inv = 1.0 / d;
        const int64_t kmax = (nmax - 1) / d;
        auto check = [&](int64_t k) {
            for (int64_t n = k * d - 1; n <= k * d + 1; ++n)
                if (n >= 0 && n < nmax && idiv((int)n, inv) != (int)(n / d)) ++bad;
        };
        for (int64_t k = 0; k < 300 && k <= kmax; ++k) check(k);
        for (int64_t k = kmax > 300 ? kmax - 300 : 0; k <= kmax + 1; ++k) check(k);
        for (int64_t j = 1; j <= 200; ++j) check(kmax * j / 201);
    }
    return bad;
}
