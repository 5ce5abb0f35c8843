// eigs.hip -- low modes of the Wilson kernel H_W and their use in deflating
// the sign function of the overlap operator (GWU-code computes the low
// eigensystem it deflates with, Sections 1 and 3 and the performance section).
//
// Eigensolver: Chebyshev-filtered subspace iteration on H_W^2 in FP64 for a
// block of m vectors.  Each pass applies T_k(Y) with Y = (2 H_W^2 / s - 1 - a)
// / (1 - a), which damps the spectrum of H_W^2 / s inside [a, 1] and amplifies
// what lies below a (the same Clenshaw machinery as the sign function), then
// orthonormalises the block (Lowdin, twice) and takes Ritz pairs of H_W itself
// from the m x m matrix V^dagger H_W V.  The small dense problems are solved on
// the host by complex Jacobi rotations; every lattice-sized operation runs on
// the GPU (broadcast dot products, complex block rotations, H_W).
//
// Deflation: with nev orthonormal eigenvectors xi_i of H_W (eigenvalues
// lambda_i), eps(H_W) v = sum_i sign(lambda_i) xi_i <xi_i, v>
//                        + eps_poly(H_W) (v - sum_i xi_i <xi_i, v>).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "wl_host.h"

namespace wl {
wl_status check_gauge(wl_gauge U);
wl_status check_field(const void *p, wl_gauge U, int nrhs, const char *what);

using zc = std::complex<double>;

// ------------------------------------------------------------------ small dense Hermitian algebra (host)

// Eigen-decomposition of a Hermitian m x m matrix (row-major) by cyclic
// complex Jacobi rotations: A = Q diag(w) Q^dagger, columns of Q the vectors.
static void herm_eig(int m, std::vector<zc> A, std::vector<double> &w, std::vector<zc> &Q)
{
    Q.assign((size_t)m * m, zc(0, 0));
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    auto at = [&](int i, int j) -> zc & { return A[(size_t)i * m + j]; };
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, diag = 0;
        for (int i = 0; i < m; ++i) {
            diag += std::norm(at(i, i));
            for (int j = i + 1; j < m; ++j) off += std::norm(at(i, j));
        }
        if (off <= 1e-32 * (diag + 1e-300)) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const zc c = at(p, q);
                const double ac = std::abs(c);
                if (ac < 1e-300) continue;
                // phase: D = diag(1, conj(ph)) on (p, q) makes A_pq real and positive
                const zc ph = c / ac;
                for (int j = 0; j < m; ++j) at(q, j) *= ph;
                for (int i = 0; i < m; ++i) at(i, q) *= std::conj(ph);
                for (int i = 0; i < m; ++i) Q[(size_t)i * m + q] *= std::conj(ph);
                // real Jacobi rotation that zeroes the (now real) pair
                const double a = at(p, p).real(), b = at(q, q).real();
                const double th = (b - a) / (2.0 * ac);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int i = 0; i < m; ++i) {  // columns
                    const zc xp = at(i, p), xq = at(i, q);
                    at(i, p) = cs * xp - sn * xq;
                    at(i, q) = sn * xp + cs * xq;
                }
                for (int j = 0; j < m; ++j) {  // rows
                    const zc xp = at(p, j), xq = at(q, j);
                    at(p, j) = cs * xp - sn * xq;
                    at(q, j) = sn * xp + cs * xq;
                }
                for (int i = 0; i < m; ++i) {
                    const zc xp = Q[(size_t)i * m + p], xq = Q[(size_t)i * m + q];
                    Q[(size_t)i * m + p] = cs * xp - sn * xq;
                    Q[(size_t)i * m + q] = sn * xp + cs * xq;
                }
            }
    }
    w.resize(m);
    for (int i = 0; i < m; ++i) w[i] = at(i, i).real();
}

// herm_eig with the eigenvalues in ascending order (columns of Q permuted alike)
static void herm_eig_sorted(int m, const std::vector<zc> &A, std::vector<double> &w, std::vector<zc> &Q)
{
    std::vector<double> w0;
    std::vector<zc> Q0;
    herm_eig(m, A, w0, Q0);
    std::vector<int> o(m);
    std::iota(o.begin(), o.end(), 0);
    std::sort(o.begin(), o.end(), [&](int x, int y) { return w0[x] < w0[y]; });
    w.resize(m);
    Q.resize((size_t)m * m);
    for (int k = 0; k < m; ++k) {
        w[k] = w0[o[k]];
        for (int i = 0; i < m; ++i) Q[(size_t)i * m + k] = Q0[(size_t)i * m + o[k]];
    }
}

// ------------------------------------------------------------------ block operations on a single-system set

// view of vector i of a field of a single-system set
static Field vec_view(const ExecSet &S, const Field &f, int i)
{
    const int stride = S.systems[0].g->geom.stride;
    Field v = f;
    v.p = (char *)f.p + (size_t)i * stride * nchunks(f.prec) * chunk_bytes(f.prec);
    v.n = f.n ? f.n + (size_t)i * stride : nullptr;
    return v;
}

// G[j][v] = <X_j, Y_v> over both parities for the vectors j of set SX and v of
// set SY (same lattice); host result, nx x ny complex, row-major by j
static wl_status block_dots(ExecSet &SX, const Field X[2], int nx, ExecSet &SY, const Field Y[2], int prec,
                            std::vector<zc> &G, hipStream_t s)
{
    const int ny = SY.nvec;
    double *d = nullptr;
    WL_TRY(SY.buffer("blk_dots", sizeof(double) * 2 * (size_t)nx * ny, (void **)&d));
    for (int j = 0; j < nx; ++j)
        for (int p = 0; p < 2; ++p) {
            const Field f[2] = {vec_view(SX, X[p], j), Y[p]};
            WL_TRY(blas(SY, BL_CDOT, prec, f, 2, nullptr,
                        red_spec(SY, p == 0 ? RED_CSTORE : RED_CACCUM, d + 2 * (size_t)ny * j, 2), s, true, 0, 1));
        }
    std::vector<double> h(2 * (size_t)nx * ny);
    WL_HIP(hipMemcpyAsync(h.data(), d, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    WL_HIP(hipStreamSynchronize(s));
    G.resize((size_t)nx * ny);
    for (size_t k = 0; k < G.size(); ++k) G[k] = zc(h[2 * k], h[2 * k + 1]);
    return WL_OK;
}

// Y_v = sum_j T[j][v] X_j (both parities), T host m x m row-major by j
static wl_status block_rotate(ExecSet &S, const Field Y[2], const Field X[2], const std::vector<zc> &T, int prec,
                              hipStream_t s)
{
    const int m = S.nvec;
    double *d = nullptr;
    WL_TRY(S.buffer("blk_rot", sizeof(double) * 2 * (size_t)m * m, (void **)&d));
    std::vector<double> h(2 * (size_t)m * m);
    // device layout T[j + m v]
    for (int j = 0; j < m; ++j)
        for (int v = 0; v < m; ++v) {
            h[2 * ((size_t)j + (size_t)m * v)] = T[(size_t)j * m + v].real();
            h[2 * ((size_t)j + (size_t)m * v) + 1] = T[(size_t)j * m + v].imag();
        }
    WL_HIP(hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
    for (int p = 0; p < 2; ++p) {
        const Field f[2] = {Y[p], X[p]};
        WL_TRY(blas(S, BL_ROT, prec, f, 2, d, no_red(), s, false));
    }
    WL_HIP(hipStreamSynchronize(s));  // h is released on return
    return WL_OK;
}

// V <- V G^{-1/2} with G = V^dagger V (Lowdin), through the scratch field T
static wl_status orthonormalise(ExecSet &S, Field V[2], Field T[2], int prec, hipStream_t s)
{
    const int m = S.nvec;
    std::vector<zc> G, Q, X((size_t)m * m);
    std::vector<double> w;
    WL_TRY(block_dots(S, V, m, S, V, prec, G, s));
    herm_eig(m, G, w, Q);
    const double wmax = *std::max_element(w.begin(), w.end());
    for (int i = 0; i < m; ++i)
        if (!(w[i] > 1e-28 * wmax)) return set_error(WL_ERR_NONFINITE, "eigensolver block lost rank");
    // X = Q diag(w^-1/2) Q^dagger
    for (int j = 0; j < m; ++j)
        for (int v = 0; v < m; ++v) {
            zc acc = 0;
            for (int k = 0; k < m; ++k) acc += Q[(size_t)j * m + k] * (1.0 / std::sqrt(w[k])) * std::conj(Q[(size_t)v * m + k]);
            X[(size_t)j * m + v] = acc;
        }
    WL_TRY(block_rotate(S, T, V, X, prec, s));
    std::swap(V[0], T[0]);
    std::swap(V[1], T[1]);
    return WL_OK;
}

// ------------------------------------------------------------------ deflation

wl_status defl_load(wl_gauge U, double kappa, int nev, const double *evecs, const double *evals, hipStream_t s,
                    Deflation *D)
{
    D->nev = nev;
    if (nev <= 0) return WL_OK;
    WL_TRY(get_set({SysEntry{U, nev, kappa}}, &D->E));
    std::fill(D->E->h_active.begin(), D->E->h_active.end(), 1);
    WL_TRY(D->E->upload_active(s));
    D->lam.assign(evals, evals + nev);
    const double *c[1] = {evecs};
    for (int p = 0; p < 2; ++p) {
        WL_TRY(D->E->field("defl_xi64_" + std::to_string(p), P_F64, &D->f64[p]));
        WL_TRY(D->E->field("defl_xi32_" + std::to_string(p), P_F32, &D->f32[p]));
        WL_TRY(pack(*D->E, c, p, D->f64[p], s));
        WL_TRY(pack(*D->E, c, p, D->f32[p], s));
    }
    return WL_OK;
}

wl_status defl_coeffs(ExecSet &S, const Deflation &D, int prec, const Field in[2], std::vector<zc> &c, hipStream_t s)
{
    const Field *xi = prec == P_F64 ? D.f64 : D.f32;
    return block_dots(*D.E, xi, D.nev, S, in, prec, c, s);
}

wl_status defl_axpy(ExecSet &S, const Deflation &D, int prec, const Field y[2], const std::vector<zc> &z, bool g5,
                    hipStream_t s)
{
    const int nv = S.nvec;
    const Field *xi = prec == P_F64 ? D.f64 : D.f32;
    double *d = nullptr;
    WL_TRY(S.buffer("defl_z", sizeof(double) * 2 * (size_t)D.nev * nv, (void **)&d));
    std::vector<double> h(2 * (size_t)D.nev * nv);
    for (size_t k = 0; k < z.size(); ++k) {
        h[2 * k] = z[k].real();
        h[2 * k + 1] = z[k].imag();
    }
    WL_HIP(hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
    for (int i = 0; i < D.nev; ++i)
        for (int p = 0; p < 2; ++p) {
            const Field f[2] = {y[p], vec_view(*D.E, xi[p], i)};
            WL_TRY(blas(S, g5 ? BL_CAXPY_G5 : BL_CAXPY, prec, f, 2, d + 2 * (size_t)nv * i, no_red(), s, true, 0, 2));
        }
    WL_HIP(hipStreamSynchronize(s));  // h is released on return
    return WL_OK;
}

}  // namespace wl

using namespace wl;

extern "C" {

wl_status wl_hw_eigs(wl_gauge U, double rho, int32_t nev, int32_t nblock, int32_t degree, double tol,
                     int32_t maxiter, double scale, double *evecs, double *evals, double *resid, int32_t *iters,
                     void *stream)
{
    clear_error();
    WL_TRY(check_gauge(U));
    if (!(rho > 0 && rho < 4)) return set_error(WL_ERR_ARG, "rho must be in (0, 4)");
    if (nev < 1 || nblock < nev || nblock > 64) return set_error(WL_ERR_ARG, "need 1 <= nev <= nblock <= 64");
    if (degree < 1 || degree > 1000) return set_error(WL_ERR_ARG, "degree must be in [1, 1000]");
    if (!(tol > 0) || maxiter < 1) return set_error(WL_ERR_ARG, "tol > 0 and maxiter >= 1 required");
    if (!std::isfinite(scale)) return set_error(WL_ERR_ARG, "scale must be finite");
    if (!evals || !resid) return set_error(WL_ERR_ARG, "null host result array");
    WL_TRY(check_field(evecs, U, nev, "evecs"));
    hipStream_t s = (hipStream_t)stream;
    const double kappa = 1.0 / (8.0 - 2.0 * rho);
    const int m = nblock;
    ExecSet *B = nullptr;
    WL_TRY(get_set({SysEntry{U, m, kappa}}, &B));
    std::fill(B->h_active.begin(), B->h_active.end(), 1);
    WL_TRY(B->upload_active(s));
    Field V[2], W[2], T[2];
    for (int p = 0; p < 2; ++p) {
        WL_TRY(B->field("eig_v" + std::to_string(p), P_F64, &V[p]));
        WL_TRY(B->field("eig_w" + std::to_string(p), P_F64, &W[p]));
        WL_TRY(B->field("eig_t" + std::to_string(p), P_F64, &T[p]));
        WL_TRY(blas(*B, BL_FILL, P_F64, &V[p], 1, nullptr, no_red(), s));
    }
    const int recon = 18;
    if (!(scale > 0)) {
        Field u[2];
        ExecSet *S1 = nullptr;
        WL_TRY(get_set({SysEntry{U, 1, kappa}}, &S1));
        std::fill(S1->h_active.begin(), S1->h_active.end(), 1);
        WL_TRY(S1->upload_active(s));
        for (int p = 0; p < 2; ++p) {
            WL_TRY(S1->field("pw_u" + std::to_string(p), P_F64, &u[p]));
            const Field f[2] = {u[p], vec_view(*B, V[p], 0)};
            WL_TRY(blas(*S1, BL_COPY, P_F64, f, 2, nullptr, no_red(), s, true, 0, 2));
        }
        double lm = 0;
        WL_TRY(power_lmax(*S1, rho, recon, 100, u, &lm, s));
        scale = 1.02 * lm;
        if (!(scale > 0)) return set_error(WL_ERR_NONFINITE, "power iteration gave %g", lm);
    }
    const double *hw_row = nullptr;
    WL_TRY(coef_table(*B, {4.0 - rho, 0, 0, 0, -0.5}, &hw_row));
    WL_TRY(orthonormalise(*B, V, T, P_F64, s));
    std::vector<double> theta(m, 0.0), res(m, 1e300);
    std::vector<int> order(m);
    double a = 0.05;  // filter window [a, 1] of H_W^2 / s
    int it = 0;
    for (; it < maxiter; ++it) {
        // filter: V <- T_degree(Y) V, the only nonzero Chebyshev coefficient at index `degree`
        SignPlan P;
        {
            const int N = degree + 1;
            const double ay = 2.0 / ((1.0 - a) * scale), by = -(1.0 + a) / (1.0 - a);
            std::vector<double> tab;
            tab.insert(tab.end(), {4.0 - rho, 0, 0, 0, -0.5});
            for (int j = 1; j < N; ++j)
                tab.insert(tab.end(), {2 * ay * (4.0 - rho), 2 * by, -1.0, j == degree ? 1.0 : 0.0, -ay});
            tab.insert(tab.end(), {ay * (4.0 - rho), by, -1.0, 0.0, -0.5 * ay});
            P.N = N;
            P.m = 4.0 - rho;
            P.rs = 1.0 / std::sqrt(scale);
            WL_TRY(coef_table(*B, tab, &P.tab));
        }
        Field y[2];
        WL_TRY(sign_poly(*B, P_F64, recon, P, V, y, s));
        for (int p = 0; p < 2; ++p) {
            const Field f[2] = {V[p], y[p]};
            WL_TRY(blas(*B, BL_COPY, P_F64, f, 2, nullptr, no_red(), s));
        }
        WL_TRY(orthonormalise(*B, V, T, P_F64, s));
        WL_TRY(orthonormalise(*B, V, T, P_F64, s));
        // Rayleigh-Ritz with H_W^2 (the wanted end of its spectrum is extreme, so
        // no spurious interior Ritz values): W = H_W V, S2 = W^dagger W ascending
        WL_TRY(apply_hw(*B, P_F64, recon, W, V, hw_row, nullptr, s));
        std::vector<zc> S2, Q;
        std::vector<double> t2;
        WL_TRY(block_dots(*B, W, m, *B, W, P_F64, S2, s));
        for (int j = 0; j < m; ++j)
            for (int v = j; v < m; ++v) {
                const zc h = 0.5 * (S2[(size_t)j * m + v] + std::conj(S2[(size_t)v * m + j]));
                S2[(size_t)j * m + v] = h;
                S2[(size_t)v * m + j] = std::conj(h);
            }
        herm_eig_sorted(m, S2, t2, Q);
        // then H_W itself on the span of the nev lowest: its Ritz pairs there are the output
        std::vector<zc> Hs;
        WL_TRY(block_dots(*B, V, m, *B, W, P_F64, Hs, s));  // V^dagger H_W V in the old basis
        {
            // H in the H^2-Ritz basis: Q^dagger Hs Q, restricted to the first nev columns
            std::vector<zc> Hn((size_t)nev * nev, zc(0, 0));
            for (int i = 0; i < nev; ++i)
                for (int k = 0; k < nev; ++k) {
                    zc acc = 0;
                    for (int j = 0; j < m; ++j)
                        for (int v = 0; v < m; ++v)
                            acc += std::conj(Q[(size_t)j * m + i]) * Hs[(size_t)j * m + v] * Q[(size_t)v * m + k];
                    Hn[(size_t)i * nev + k] = acc;
                }
            for (int i = 0; i < nev; ++i)
                for (int k = i; k < nev; ++k) {
                    const zc h = 0.5 * (Hn[(size_t)i * nev + k] + std::conj(Hn[(size_t)k * nev + i]));
                    Hn[(size_t)i * nev + k] = h;
                    Hn[(size_t)k * nev + i] = std::conj(h);
                }
            std::vector<double> th;
            std::vector<zc> Qh;
            herm_eig_sorted(nev, Hn, th, Qh);
            // total rotation: Q then blockdiag(Qh, 1) on the first nev columns
            std::vector<zc> R((size_t)m * m, zc(0, 0));
            for (int j = 0; j < m; ++j) {
                for (int k = 0; k < nev; ++k) {
                    zc acc = 0;
                    for (int i = 0; i < nev; ++i) acc += Q[(size_t)j * m + i] * Qh[(size_t)i * nev + k];
                    R[(size_t)j * m + k] = acc;
                }
                for (int k = nev; k < m; ++k) R[(size_t)j * m + k] = Q[(size_t)j * m + k];
            }
            for (int k = 0; k < m; ++k) theta[k] = k < nev ? th[k] : std::sqrt(std::max(t2[k], 0.0));
            Q.swap(R);
        }
        WL_TRY(block_rotate(*B, T, V, Q, P_F64, s));
        std::swap(V[0], T[0]);
        std::swap(V[1], T[1]);
        WL_TRY(block_rotate(*B, T, W, Q, P_F64, s));
        std::swap(W[0], T[0]);
        std::swap(W[1], T[1]);
        // residuals |W_v - theta_v V_v| of the Ritz pairs, formed explicitly in T
        double *d = nullptr, *z = nullptr;
        WL_TRY(B->buffer("eig_norm", sizeof(double) * m, (void **)&d));
        WL_TRY(B->buffer("eig_theta", sizeof(double) * 2 * m, (void **)&z));
        std::vector<double> hz(2 * m, 0.0);
        for (int v = 0; v < m; ++v) hz[2 * v] = -theta[v];
        WL_HIP(hipMemcpyAsync(z, hz.data(), sizeof(double) * 2 * m, hipMemcpyHostToDevice, s));
        for (int p = 0; p < 2; ++p) {
            const Field fc[2] = {T[p], W[p]};
            WL_TRY(blas(*B, BL_COPY, P_F64, fc, 2, nullptr, no_red(), s, false));
            const Field fa[2] = {T[p], V[p]};
            WL_TRY(blas(*B, BL_CAXPY, P_F64, fa, 2, z, no_red(), s, false));
            WL_TRY(blas(*B, BL_NORM2, P_F64, &T[p], 1, nullptr, red_spec(*B, p == 0 ? RED_STORE : RED_ACCUM, d), s,
                        false));
        }
        std::vector<double> n2(m);
        WL_HIP(hipMemcpyAsync(n2.data(), d, sizeof(double) * m, hipMemcpyDeviceToHost, s));
        WL_HIP(hipStreamSynchronize(s));
        for (int v = 0; v < m; ++v) res[v] = std::sqrt(std::max(n2[v], 0.0));
        // the wanted pairs are vectors 0..nev-1, ordered by |theta|
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.begin() + nev,
                  [&](int x, int y2) { return std::fabs(theta[x]) < std::fabs(theta[y2]); });
        bool ok = true;
        double worst = 0;
        for (int i = 0; i < nev; ++i) {
            ok = ok && res[order[i]] <= tol;
            worst = std::max(worst, res[order[i]]);
        }
        if (getenv("WL_DEBUG"))
            fprintf(stderr, "[wl eigs] pass %d: window a = %.3e, worst wanted residual %.3e, |theta| %.4e .. %.4e\n", it,
                    a, worst, std::fabs(theta[order[0]]), std::fabs(theta[order[nev - 1]]));
        if (ok) {
            ++it;
            break;
        }
        // the next filter damps everything above the block's largest H_W^2 Ritz value
        a = std::min(0.9, std::max(1e-4, t2[m - 1] / scale));
    }
    // the nev Ritz vectors of smallest |theta|, in that order, are vectors 0..nev-1 of T
    std::vector<zc> sel((size_t)m * m, zc(0, 0));
    for (int i = 0; i < nev; ++i) sel[(size_t)order[i] * m + i] = 1.0;
    WL_TRY(block_rotate(*B, T, V, sel, P_F64, s));
    ExecSet *E = nullptr;
    WL_TRY(get_set({SysEntry{U, nev, kappa}}, &E));
    Field Ef[2];
    double *out[1] = {evecs};
    for (int p = 0; p < 2; ++p) {
        WL_TRY(E->field("eig_out" + std::to_string(p), P_F64, &Ef[p]));
        const size_t bytes = (size_t)nev * U->geom.stride * nchunks(P_F64) * chunk_bytes(P_F64);
        WL_HIP(hipMemcpyAsync(Ef[p].p, T[p].p, bytes, hipMemcpyDeviceToDevice, s));
        WL_TRY(unpack(*E, out, p, Ef[p], s));
    }
    WL_HIP(hipStreamSynchronize(s));
    bool ok = true;
    for (int i = 0; i < nev; ++i) {
        evals[i] = theta[order[i]];
        resid[i] = res[order[i]];
        ok = ok && resid[i] <= tol;
    }
    if (iters) *iters = it;
    if (!ok) return set_error(WL_ERR_NOCONV, "eigenpairs not converged to %g in %d passes", tol, maxiter);
    return WL_OK;
}

}  // extern "C"
