// clover.hip -- the Sheikholeslami-Wohlert clover term of the Wilson-clover
// operator (QUDA_DIRAC_CLOVER of Table 1), built on the GPU from the canonical
// FP64 links once per (gauge field, kappa c_sw):
//
//   Q_mn(x) = the four plaquettes of the m-n plane with a corner at x, each a
//             closed loop from x, m-direction first
//   F_mn(x) = (Q_mn(x) - Q_mn(x)^dagger) / 8
//   A(x)    = 1 + i kappa c_sw sum_{m<n} s_mn F_mn(x),   s_mn = (i/2)[g_m, g_n]
//
// so that D = A - kappa H (the hopping term of wl_core.h).  A commutes with g5
// and is stored as two packed Hermitian 6x6 blocks per site (wl_core.h); the
// inverse of each block comes from Gauss-Jordan elimination with partial
// pivoting in FP64.  Gauge links are periodic; the fermion boundary sign of
// the hop does not enter the loops.
#include "wl_kernels.h"

namespace wl {

namespace {

using C = cpx<double>;

__device__ __forceinline__ C cm(C a, C b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// DeGrand-Rossi gamma_mu entry (i, j)
__device__ C gamma_entry(int mu, int i, int j)
{
    switch (mu) {
    case 0:  // gx: (0,3) = i, (1,2) = i, (2,1) = -i, (3,0) = -i
        if (i + j != 3) return {0, 0};
        return {0.0, i < 2 ? 1.0 : -1.0};
    case 1:  // gy: (0,3) = -1, (1,2) = 1, (2,1) = 1, (3,0) = -1
        if (i + j != 3) return {0, 0};
        return {(i == 0 || i == 3) ? -1.0 : 1.0, 0.0};
    case 2:  // gz: (0,2) = i, (1,3) = -i, (2,0) = -i, (3,1) = i
        if ((i ^ j) != 2) return {0, 0};
        return {0.0, (i == 0 || i == 3) ? 1.0 : -1.0};
    default:  // gt: (0,2) = (1,3) = (2,0) = (3,1) = 1
        if ((i ^ j) != 2) return {0, 0};
        return {1.0, 0.0};
    }
}

// s_mn (i, j) = (i/2) (g_m g_n - g_n g_m)(i, j)
__device__ C sigma_entry(int m, int n, int i, int j)
{
    C v{0, 0};
    for (int k = 0; k < 4; ++k) {
        const C a = cm(gamma_entry(m, i, k), gamma_entry(n, k, j));
        const C b = cm(gamma_entry(n, i, k), gamma_entry(m, k, j));
        v.re += a.re - b.re;
        v.im += a.im - b.im;
    }
    return {-0.5 * v.im, 0.5 * v.re};
}

struct M3 {
    C e[9];
};

__device__ __forceinline__ M3 load_u(const double *U, long site, int mu)
{
    const double2 *p = (const double2 *)U + (site * 4 + mu) * 9;
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 w = p[k];
        m.e[k] = {w.x, w.y};
    }
    return m;
}

// c = op(a) op(b), op = dagger when the flag is set
__device__ M3 mul(const M3 &a, bool ad, const M3 &b, bool bd)
{
    M3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            C v{0, 0};
            for (int k = 0; k < 3; ++k) {
                C x = ad ? C{a.e[k * 3 + i].re, -a.e[k * 3 + i].im} : a.e[i * 3 + k];
                C y = bd ? C{b.e[j * 3 + k].re, -b.e[j * 3 + k].im} : b.e[k * 3 + j];
                const C p = cm(x, y);
                v.re += p.re;
                v.im += p.im;
            }
            c.e[i * 3 + j] = v;
        }
    return c;
}

__device__ long site_of(const SysDesc &d, const int c[4])
{
    return c[0] + (long)d.L[0] * (c[1] + (long)d.L[1] * (c[2] + (long)d.L[2] * c[3]));
}

__device__ long shifted(const SysDesc &d, const int c[4], int m, int a, int n, int b)
{
    int y[4] = {c[0], c[1], c[2], c[3]};
    y[m] = (y[m] + a + d.L[m]) % d.L[m];
    y[n] = (y[n] + b + d.L[n]) % d.L[n];
    return site_of(d, y);
}

// the clover-leaf field strength F_mn at site s
__device__ M3 field_strength(const double *U, const SysDesc &d, long s, const int c[4], int m, int n)
{
    const long xm = shifted(d, c, m, 1, n, 0), xn = shifted(d, c, m, 0, n, 1);
    const long xmm = shifted(d, c, m, -1, n, 0), xnm = shifted(d, c, m, 0, n, -1);
    const long xmm_np = shifted(d, c, m, -1, n, 1), xmm_nm = shifted(d, c, m, -1, n, -1);
    const long xmp_nm = shifted(d, c, m, 1, n, -1);
    M3 Q;
    for (int k = 0; k < 9; ++k) Q.e[k] = {0, 0};
    auto add = [&Q](const M3 &l) {
        for (int k = 0; k < 9; ++k) {
            Q.e[k].re += l.e[k].re;
            Q.e[k].im += l.e[k].im;
        }
    };
    // x -> x+m -> x+m+n -> x+n -> x:   U_m(x) U_n(x+m) U_m(x+n)^+ U_n(x)^+
    add(mul(mul(mul(load_u(U, s, m), false, load_u(U, xm, n), false), false, load_u(U, xn, m), true), false,
            load_u(U, s, n), true));
    // x -> x+n -> x+n-m -> x-m -> x:   U_n(x) U_m(x+n-m)^+ U_n(x-m)^+ U_m(x-m)
    add(mul(mul(mul(load_u(U, s, n), false, load_u(U, xmm_np, m), true), false, load_u(U, xmm, n), true), false,
            load_u(U, xmm, m), false));
    // x -> x-m -> x-m-n -> x-n -> x:   U_m(x-m)^+ U_n(x-m-n)^+ U_m(x-m-n) U_n(x-n)
    add(mul(mul(mul(load_u(U, xmm, m), true, load_u(U, xmm_nm, n), true), false, load_u(U, xmm_nm, m), false),
            false, load_u(U, xnm, n), false));
    // x -> x-n -> x-n+m -> x+m -> x:   U_n(x-n)^+ U_m(x-n) U_n(x-n+m) U_m(x)^+
    add(mul(mul(mul(load_u(U, xnm, n), true, load_u(U, xnm, m), false), false, load_u(U, xmp_nm, n), false), false,
            load_u(U, s, m), true));
    M3 F;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            F.e[i * 3 + j] = {(Q.e[i * 3 + j].re - Q.e[j * 3 + i].re) / 8.0, (Q.e[i * 3 + j].im + Q.e[j * 3 + i].im) / 8.0};
    return F;
}

// packed block b (36 reals) of the parity-major field at (par, cb)
__device__ void store_block(void *A64, void *A32, void *A16, const SysDesc &d, int par, int cb, int b,
                            const double m[36])
{
    double2 *f64 = (double2 *)clover_parity<P_F64>(A64, par, d.stride);
    for (int k = 0; k < 18; ++k) f64[(size_t)(18 * b + k) * d.stride + cb] = double2{m[2 * k], m[2 * k + 1]};
    float4 *f32 = (float4 *)clover_parity<P_F32>(A32, par, d.stride);
    for (int k = 0; k < 9; ++k)
        f32[(size_t)(9 * b + k) * d.stride + cb] =
            float4{(float)m[4 * k], (float)m[4 * k + 1], (float)m[4 * k + 2], (float)m[4 * k + 3]};
    // FP16: block b is the 8-byte units 9b .. 9b + 8 of the site's 18 (two per
    // 16-byte row), so the two blocks of a site, written by different threads,
    // never share a store
    char *f16 = (char *)clover_parity<P_F16>(A16, par, d.stride);
    for (int k = 0; k < 9; ++k) {
        const int u = 9 * b + k;
        const uint2 w{pack2_d<P_F16>(m[4 * k], m[4 * k + 1]), pack2_d<P_F16>(m[4 * k + 2], m[4 * k + 3])};
        *(uint2 *)(f16 + ((size_t)(u >> 1) * d.stride + cb) * 16 + (u & 1) * 8) = w;
    }
}

__global__ __launch_bounds__(256) void k_clover_build(const double *U, SysDesc d, double kc, void *A64, void *A32,
                                                      void *A16)
{
    const long V = 2L * d.Vh;
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    int c[4];
    long r = s;
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(r % d.L[mu]);
        r /= d.L[mu];
    }
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    const int cb = (int)(s >> 1);
    double m[2][36];
    for (int b = 0; b < 2; ++b) {
        for (int k = 0; k < 36; ++k) m[b][k] = 0.0;
        for (int k = 0; k < 6; ++k) m[b][k] = 1.0;
    }
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll 1
        for (int nu = mu + 1; nu < 4; ++nu) {
            const M3 F = field_strength(U, d, s, c, mu, nu);
            for (int b = 0; b < 2; ++b)
                for (int i2 = 0; i2 < 2; ++i2)
                    for (int j2 = 0; j2 < 2; ++j2) {
                        const C sg = sigma_entry(mu, nu, 2 * b + i2, 2 * b + j2);
                        if (sg.re == 0.0 && sg.im == 0.0) continue;
                        // i kc s F: entry (3 i2 + a, 3 j2 + e)
                        const C f = {-kc * sg.im, kc * sg.re};
                        for (int a = 0; a < 3; ++a)
                            for (int e = 0; e < 3; ++e) {
                                const int row = 3 * i2 + a, col = 3 * j2 + e;
                                if (row > col) continue;
                                const C v = cm(f, F.e[a * 3 + e]);
                                if (row == col) {
                                    m[b][row] += v.re;
                                } else {
                                    const int u = clov_upper(row, col);
                                    m[b][u] += v.re;
                                    m[b][u + 1] += v.im;
                                }
                            }
                    }
        }
    store_block(A64, A32, A16, d, par, cb, 0, m[0]);
    store_block(A64, A32, A16, d, par, cb, 1, m[1]);
}

// one thread per (site, block): the inverse of a Hermitian 6x6 block
__global__ __launch_bounds__(256) void k_clover_invert(SysDesc d, const void *A64, void *Ainv64, void *Ainv32,
                                                       void *Ainv16)
{
    const long n = 2L * 2L * d.Vh;  // (parity, cb, block)
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int b = (int)(t & 1);
    const long pc = t >> 1;
    const int par = (int)(pc / d.Vh), cb = (int)(pc % d.Vh);
    const double2 *f64 = (const double2 *)clover_parity<P_F64>(A64, par, d.stride);
    double p[36];
    for (int k = 0; k < 18; ++k) {
        const double2 w = f64[(size_t)(18 * b + k) * d.stride + cb];
        p[2 * k] = w.x;
        p[2 * k + 1] = w.y;
    }
    C a[6][12];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 12; ++j) a[i][j] = {0, 0};
    for (int i = 0; i < 6; ++i) {
        a[i][i] = {p[i], 0.0};
        a[i][6 + i] = {1.0, 0.0};
        for (int j = i + 1; j < 6; ++j) {
            const int u = clov_upper(i, j);
            a[i][j] = {p[u], p[u + 1]};
            a[j][i] = {p[u], -p[u + 1]};
        }
    }
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        double best = a[col][col].re * a[col][col].re + a[col][col].im * a[col][col].im;
        for (int r = col + 1; r < 6; ++r) {
            const double v = a[r][col].re * a[r][col].re + a[r][col].im * a[r][col].im;
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (piv != col)
            for (int j = 0; j < 12; ++j) {
                const C tmp = a[col][j];
                a[col][j] = a[piv][j];
                a[piv][j] = tmp;
            }
        const C dv = a[col][col];
        const double den = dv.re * dv.re + dv.im * dv.im;
        const C inv = {dv.re / den, -dv.im / den};  // a singular block gives non-finite entries
        for (int j = 0; j < 12; ++j) a[col][j] = cm(a[col][j], inv);
        for (int r = 0; r < 6; ++r) {
            if (r == col) continue;
            const C f = a[r][col];
            for (int j = 0; j < 12; ++j) {
                const C q = cm(f, a[col][j]);
                a[r][j].re -= q.re;
                a[r][j].im -= q.im;
            }
        }
    }
    // the inverse of a Hermitian matrix is Hermitian: keep its upper triangle
    double q[36];
    for (int i = 0; i < 6; ++i) {
        q[i] = a[i][6 + i].re;
        for (int j = i + 1; j < 6; ++j) {
            const int u = clov_upper(i, j);
            q[u] = a[i][6 + j].re;
            q[u + 1] = a[i][6 + j].im;
        }
    }
    store_block(Ainv64, Ainv32, Ainv16, d, par, cb, b, q);
}

}  // namespace

hipError_t launch_clover_build(const double *U_canon, const SysDesc &d, double kc, void *A64, void *A32, void *A16,
                               hipStream_t s)
{
    const long V = 2L * d.Vh;
    hipLaunchKernelGGL(k_clover_build, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, U_canon, d, kc, A64, A32,
                       A16);
    return hipGetLastError();
}

hipError_t launch_clover_invert(const SysDesc &d, const void *A64, void *Ainv64, void *Ainv32, void *Ainv16,
                                hipStream_t s)
{
    const long n = 4L * d.Vh;
    hipLaunchKernelGGL(k_clover_invert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, A64, Ainv64, Ainv32,
                       Ainv16);
    return hipGetLastError();
}

}  // namespace wl
