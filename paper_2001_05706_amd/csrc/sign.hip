// sign.hip -- Chebyshev approximation of the sign function of the Wilson
// kernel H_W = g5 D_m(-rho), the inner kernel of the overlap operator that
// GWU-code inverts (Sections 1 and 3):
//   eps(H_W) v ~= s^{-1/2} H_W p(H_W^2 / s) v,
// p the degree-d interpolant of x^{-1/2} on [lo, hi] at the d+1 first-kind
// Chebyshev nodes, applied with the Clenshaw recurrence.  Each recurrence step
// is two whole-lattice H_W applications on all right-hand sides; the second
// carries the recurrence update in its epilogue, so a step costs four hop
// launches (two per parity) and no separate vector kernels.
#include <cmath>
#include <vector>

#include "wl_host.h"

namespace wl {
wl_status check_gauge(wl_gauge U);
wl_status check_field(const void *p, wl_gauge U, int nrhs, const char *what);

// Chebyshev interpolation coefficients of x^{-1/2} on [lo, hi]:
//   theta_k = pi (k + 1/2) / N, x_k = (hi - lo)/2 cos theta_k + (hi + lo)/2,
//   c_j = (2/N) sum_k x_k^{-1/2} cos(j theta_k),  N = degree + 1.
static std::vector<double> invsqrt_coeffs(int degree, double lo, double hi)
{
    const int N = degree + 1;
    std::vector<double> th(N), fx(N), c(N);
    for (int k = 0; k < N; ++k) {
        th[k] = M_PI * (k + 0.5) / N;
        fx[k] = 1.0 / std::sqrt(0.5 * (hi - lo) * std::cos(th[k]) + 0.5 * (hi + lo));
    }
    for (int j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int k = 0; k < N; ++k) acc += fx[k] * std::cos(j * th[k]);
        c[j] = 2.0 * acc / N;
    }
    return c;
}

// H_W applied to the two parities of `in` into `out`; coef = {m a, ..., c} per system
wl_status apply_hw(ExecSet &S, int prec, int recon, const Field out[2], const Field in[2], const double *coef,
                          const RedSpec *red, hipStream_t s)
{
    Epi e[2];
    for (int p = 0; p < 2; ++p) {
        e[p].coef = coef;
        e[p].g5 = 1;
        e[p].nx = 1;
        e[p].X[0] = in[p];
    }
    if (!red) return hop2(S, prec, recon, false, out, in, e, s);
    for (int p = 0; p < 2; ++p) WL_TRY(hop(S, prec, recon, false, p, out[p], in[1 - p], e[p], red[p], s));
    return WL_OK;
}

// power iteration for lambda_max(H_W^2) on vector 0 of the set; FP64
wl_status power_lmax(ExecSet &S, double rho, int recon, int iters, const Field u[2], double *lmax,
                            hipStream_t s)
{
    Field w[2];
    WL_TRY(S.field("pw_w0", P_F64, &w[0]));
    WL_TRY(S.field("pw_w1", P_F64, &w[1]));
    std::vector<double> c;
    for (size_t i = 0; i < S.systems.size(); ++i) c.insert(c.end(), {4.0 - rho, 0, 0, 0, -0.5});
    const double *coef = nullptr;
    WL_TRY(coef_table(S, c, &coef));
    double *nw = S.scal(SC_QQ), *nu = S.scal(SC_RR);
    // normalise the start vector
    WL_TRY(blas(S, BL_NORM2, P_F64, &u[0], 1, nullptr, red_spec(S, RED_STORE, nu), s));
    WL_TRY(blas(S, BL_NORM2, P_F64, &u[1], 1, nullptr, red_spec(S, RED_ACCUM, nu), s));
    for (int p = 0; p < 2; ++p) WL_TRY(blas(S, BL_SCALE_RSQRT, P_F64, &u[p], 1, nu, no_red(), s));
    const RedSpec rw[2] = {red_spec(S, RED_STORE, nw), red_spec(S, RED_ACCUM, nw)};
    const RedSpec ru[2] = {red_spec(S, RED_STORE, nu), red_spec(S, RED_ACCUM, nu)};
    for (int it = 0; it < iters; ++it) {
        // |H_W u|^2 with |u| = 1 is the Rayleigh quotient of H_W^2
        WL_TRY(apply_hw(S, P_F64, recon, w, u, coef, rw, s));
        WL_TRY(apply_hw(S, P_F64, recon, u, w, coef, ru, s));
        for (int p = 0; p < 2; ++p) WL_TRY(blas(S, BL_SCALE_RSQRT, P_F64, &u[p], 1, nu, no_red(), s));
    }
    double h = 0;
    WL_HIP(hipMemcpyAsync(&h, nw, sizeof(double), hipMemcpyDeviceToHost, s));
    WL_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(h)) return set_error(WL_ERR_NONFINITE, "non-finite power iteration");
    *lmax = h;
    return WL_OK;
}

// 1.02 x the power-iteration estimate (100 steps) of lambda_max(H_W^2), started
// from the first canonical field of v0
wl_status hw2_scale(wl_gauge U, double rho, const double *v0, hipStream_t s, double *scale)
{
    ExecSet *S1 = nullptr;
    WL_TRY(get_set({SysEntry{U, 1, 1.0 / (8.0 - 2.0 * rho)}}, &S1));
    std::fill(S1->h_active.begin(), S1->h_active.end(), 1);
    WL_TRY(S1->upload_active(s));
    Field u[2];
    WL_TRY(S1->field("pw_u0", P_F64, &u[0]));
    WL_TRY(S1->field("pw_u1", P_F64, &u[1]));
    const double *c[1] = {v0};
    WL_TRY(pack(*S1, c, 0, u[0], s));
    WL_TRY(pack(*S1, c, 1, u[1], s));
    double lm = 0;
    WL_TRY(power_lmax(*S1, rho, 18, 100, u, &lm, s));
    *scale = 1.02 * lm;
    if (!(*scale > 0)) return set_error(WL_ERR_NONFINITE, "power iteration gave %g", lm);
    return WL_OK;
}

wl_status sign_plan(ExecSet &S, double rho, int degree, double lo, double hi, double scale, SignPlan *P)
{
    const int N = degree + 1;
    const std::vector<double> c = invsqrt_coeffs(degree, lo, hi);
    const double m = 4.0 - rho;
    const double ay = 2.0 / ((hi - lo) * scale), by = -(hi + lo) / (hi - lo);
    // coefficient rows: [0] H_W, [1..N-1] Clenshaw steps j, [N] final p v
    std::vector<double> tab;
    tab.insert(tab.end(), {m, 0, 0, 0, -0.5});
    for (int j = 1; j < N; ++j) tab.insert(tab.end(), {2 * ay * m, 2 * by, -1.0, c[j], -ay});
    tab.insert(tab.end(), {ay * m, by, -1.0, 0.5 * c[0], -0.5 * ay});
    P->N = N;
    P->m = m;
    P->rs = 1.0 / std::sqrt(scale);
    return coef_table(S, tab, &P->tab);
}

wl_status sign_poly(ExecSet &S, int prec, int recon, const SignPlan &P, const Field v[2], Field y[2], hipStream_t s)
{
    Field b[3][2], w[2];
    for (int p = 0; p < 2; ++p) {
        WL_TRY(S.field("sg_w" + std::to_string(p), prec, &w[p]));
        for (int j = 0; j < 3; ++j) WL_TRY(S.field("sg_b" + std::to_string(j) + std::to_string(p), prec, &b[j][p]));
    }
    // b_{N} = b_{N+1} = 0
    int i0 = 0, i1 = 1, i2 = 2;  // b_j, b_{j+1}, b_{j+2}
    for (int p = 0; p < 2; ++p) {
        WL_TRY(blas(S, BL_ZERO, prec, &b[i1][p], 1, nullptr, no_red(), s));
        WL_TRY(blas(S, BL_ZERO, prec, &b[i2][p], 1, nullptr, no_red(), s));
    }
    auto step = [&](const double *coef, const Field *dst) -> wl_status {
        // w = H_W b_{j+1};  dst = g5(a0 w + c hop w) + a1 b_{j+1} + a2 b_{j+2} + a3 v
        WL_TRY(apply_hw(S, prec, recon, w, b[i1], P.tab, nullptr, s));
        Epi e[2];
        for (int p = 0; p < 2; ++p) {
            e[p].coef = coef;
            e[p].g5 = 1;
            e[p].nx = 4;
            e[p].X[0] = w[p];
            e[p].X[1] = b[i1][p];
            e[p].X[2] = b[i2][p];
            e[p].X[3] = v[p];
        }
        return hop2(S, prec, recon, false, dst, w, e, s);
    };
    for (int j = P.N - 1; j >= 1; --j) {
        WL_TRY(step(P.tab + 5 * j, b[i0]));
        const int t = i2;
        i2 = i1;
        i1 = i0;
        i0 = t;
    }
    // p v = Y b_1 - b_2 + c_0 v / 2
    WL_TRY(step(P.tab + 5 * P.N, b[i0]));
    y[0] = b[i0][0];
    y[1] = b[i0][1];
    return WL_OK;
}

}  // namespace wl

using namespace wl;

extern "C" {

wl_status wl_hw2_lmax(wl_gauge U, double rho, const double *v0, int32_t iters, double *lmax, void *stream)
{
    clear_error();
    WL_TRY(check_gauge(U));
    if (!lmax) return set_error(WL_ERR_ARG, "null result pointer");
    if (!(rho > 0 && rho < 4)) return set_error(WL_ERR_ARG, "rho must be in (0, 4)");
    if (iters < 1) return set_error(WL_ERR_ARG, "iters must be >= 1");
    WL_TRY(check_field(v0, U, 1, "v0"));
    hipStream_t s = (hipStream_t)stream;
    ExecSet *S = nullptr;
    WL_TRY(get_set({SysEntry{U, 1, 1.0 / (8.0 - 2.0 * rho)}}, &S));
    std::fill(S->h_active.begin(), S->h_active.end(), 1);
    WL_TRY(S->upload_active(s));
    Field u[2];
    WL_TRY(S->field("pw_u0", P_F64, &u[0]));
    WL_TRY(S->field("pw_u1", P_F64, &u[1]));
    const double *c[1] = {v0};
    WL_TRY(pack(*S, c, 0, u[0], s));
    WL_TRY(pack(*S, c, 1, u[1], s));
    return power_lmax(*S, rho, 18, iters, u, lmax, s);
}

wl_status overlap_sign_cheb(wl_gauge U, const double *in, double *out, int32_t nrhs, double rho, int32_t degree,
                            double lo, double hi, double scale, wl_prec prec, int32_t recon, int32_t nev,
                            const double *evecs, const double *evals, void *stream)
{
    clear_error();
    if (nev < 0 || nev > 64) return set_error(WL_ERR_ARG, "nev must be in [0, 64]");
    if (nev > 0 && !evals) return set_error(WL_ERR_ARG, "null eigenvalues");
    if (nev > 0) WL_TRY(check_field(evecs, U, nev, "evecs"));
    WL_TRY(check_gauge(U));
    if (nrhs < 1) return set_error(WL_ERR_ARG, "nrhs must be >= 1");
    if (!(rho > 0 && rho < 4)) return set_error(WL_ERR_ARG, "rho must be in (0, 4)");
    if (degree < 1 || degree > 100000) return set_error(WL_ERR_ARG, "degree must be in [1, 100000]");
    if (!(lo > 0 && lo < hi) || !std::isfinite(hi)) return set_error(WL_ERR_ARG, "0 < lo < hi required");
    if (!std::isfinite(scale)) return set_error(WL_ERR_ARG, "scale must be finite");
    if (prec != WL_F64 && prec != WL_F32) return set_error(WL_ERR_PREC, "sign function runs in FP64 or FP32");
    if (!prec_recon_ok(prec, recon)) return set_error(WL_ERR_PREC, "unsupported precision %d / recon %d", prec, recon);
    WL_TRY(check_field(in, U, nrhs, "in"));
    WL_TRY(check_field(out, U, nrhs, "out"));
    const size_t bytes = (size_t)nrhs * 2 * U->geom.Vh * 24 * sizeof(double);
    if ((const char *)in < (const char *)out + bytes && (const char *)out < (const char *)in + bytes)
        return set_error(WL_ERR_ARG, "in and out overlap");
    hipStream_t s = (hipStream_t)stream;
    ExecSet *S = nullptr;
    WL_TRY(get_set({SysEntry{U, nrhs, 1.0 / (8.0 - 2.0 * rho)}}, &S));
    std::fill(S->h_active.begin(), S->h_active.end(), 1);
    WL_TRY(S->upload_active(s));
    WL_HIP(hipMemsetAsync(S->bad, 0, sizeof(int32_t) * S->nvec, s));
    const double *cin[1] = {in};
    double *cout[1] = {out};

    if (!(scale > 0)) WL_TRY(hw2_scale(U, rho, in, s, &scale));

    Deflation D;
    WL_TRY(defl_load(U, 1.0 / (8.0 - 2.0 * rho), nev, evecs, evals, s, &D));
    Field v[2], w[2], y[2];
    for (int p = 0; p < 2; ++p) {
        WL_TRY(S->field("sg_v" + std::to_string(p), prec, &v[p]));
        WL_TRY(S->field("sg_w" + std::to_string(p), prec, &w[p]));
        WL_TRY(pack(*S, cin, p, v[p], s));
    }
    // deflation: the polynomial acts on v - sum_i xi_i <xi_i, v>
    std::vector<std::complex<double>> c, z;
    if (D.nev) {
        WL_TRY(defl_coeffs(*S, D, prec, v, c, s));
        z.resize(c.size());
        for (size_t k = 0; k < c.size(); ++k) z[k] = -c[k];
        WL_TRY(defl_axpy(*S, D, prec, v, z, false, s));
    }
    SignPlan P;
    WL_TRY(sign_plan(*S, rho, degree, lo, hi, scale, &P));
    WL_TRY(sign_poly(*S, prec, recon, P, v, y, s));
    // out = s^{-1/2} H_W (p v) (+ sum_i sign(lambda_i) xi_i <xi_i, v>)
    const double *orow = nullptr;
    WL_TRY(coef_table(*S, {P.rs * P.m, 0, 0, 0, -0.5 * P.rs}, &orow));
    WL_TRY(apply_hw(*S, prec, recon, w, y, orow, nullptr, s));
    if (D.nev) {
        for (size_t k = 0; k < c.size(); ++k) z[k] = (D.lam[k / S->nvec] > 0 ? 1.0 : -1.0) * c[k];
        WL_TRY(defl_axpy(*S, D, prec, w, z, false, s));
    }
    for (int p = 0; p < 2; ++p) WL_TRY(unpack(*S, cout, p, w[p], s));
    WL_HIP(hipStreamSynchronize(s));
    return WL_OK;
}

}  // extern "C"
