// overlap.hip -- the overlap operator of GWU-code's inverter (Sections 1 and 3)
// and its solve, built on the Chebyshev sign function of sign.hip:
//
//   D_ov(m)         = (rho + m/2) + (rho - m/2) g5 eps(H_W)
//   D_ov(m)^dagger  = (rho + m/2) + (rho - m/2) eps(H_W) g5
//
// with eps(H_W) v ~= s^{-1/2} H_W p(H_W^2 / s) v.  The last H_W of the sign
// function carries the whole combination in its hop epilogue, so one operator
// application is exactly one sign-function evaluation (plus a g5 copy for the
// adjoint) with no separate vector kernels.
//
// The solve is CG on the normal equations D^dagger D x = D^dagger eta with the
// residual r = eta - D x of the original system tracked (q = D p is computed
// anyway), inside a defect-correction loop: the residual of the accumulated
// FP64 solution is recomputed with the FP64 operator, an inner CG in the
// working precision reduces it by `delta`, and its correction is added to the
// FP64 solution.  With an FP64 working precision the first inner solve goes
// straight to the tolerance.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "wl_host.h"

namespace wl {
wl_status check_gauge(wl_gauge U);
wl_status check_field(const void *p, wl_gauge U, int nrhs, const char *what);

namespace {

struct Overlap {
    ExecSet *S = nullptr;
    SignPlan P;
    int recon = 12;
    double a = 0, b = 0;  // rho + m/2, rho - m/2
    Deflation D;          // low modes of H_W treated exactly (nev = 0: none)
};

// out = alpha D v + beta1 X1 + beta2 X2 (dagger: D^dagger), both parities.
// v must not alias out; the reduction (if any) is |out|^2 over both parities
// into red_dst (STORE on parity 0, ACCUM on parity 1).
wl_status ov_apply(Overlap &O, int prec, bool dagger, const Field out[2], const Field v[2], double alpha,
                   const Field *X1, double beta1, const Field *X2, double beta2, double *red_dst, hipStream_t s)
{
    ExecSet &S = *O.S;
    Field in[2] = {v[0], v[1]};
    if (dagger || O.D.nev) {
        // eps acts on g5 v (adjoint) or on a copy that the deflation projects
        for (int p = 0; p < 2; ++p) {
            WL_TRY(S.field("ov_g5v" + std::to_string(p), prec, &in[p]));
            const Field f[2] = {in[p], v[p]};
            WL_TRY(blas(S, dagger ? BL_G5COPY : BL_COPY, prec, f, 2, nullptr, no_red(), s));
        }
    }
    std::vector<std::complex<double>> c, z;
    if (O.D.nev) {
        WL_TRY(defl_coeffs(S, O.D, prec, in, c, s));
        z.resize(c.size());
        for (size_t k = 0; k < c.size(); ++k) z[k] = -c[k];
        WL_TRY(defl_axpy(S, O.D, prec, in, z, false, s));
    }
    Field y[2];
    WL_TRY(sign_poly(S, prec, O.recon, O.P, in, y, s));
    // g5 eps u = s^{-1/2} (m y - hop(y) / 2), eps u = g5 of that:
    //   out = G5?(alpha b s^{-1/2} (m y - hop y / 2)) + alpha a v + beta1 X1 + beta2 X2
    // where the a v term must be added outside the g5: it sits in X slot 1
    const double k = alpha * O.b * O.P.rs;
    const double *row = nullptr;
    WL_TRY(coef_table(S, {k * O.P.m, alpha * O.a, beta1, beta2, -0.5 * k}, &row));
    for (int p = 0; p < 2; ++p) {
        Epi e;
        e.coef = row;
        e.g5 = dagger ? 1 : 0;
        e.nx = X2 ? 4 : (X1 ? 3 : 2);
        e.X[0] = y[p];
        e.X[1] = v[p];
        if (X1) e.X[2] = X1[p];
        if (X2) e.X[3] = X2[p];
        // with deflation the norm is taken after the exact low-mode part is added
        const RedSpec r = red_dst && !O.D.nev ? red_spec(S, p == 0 ? RED_STORE : RED_ACCUM, red_dst) : no_red();
        WL_TRY(hop(S, prec, O.recon, false, p, out[p], y[1 - p], e, r, s));
    }
    if (O.D.nev) {
        // + alpha b (g5) sum_i sign(lambda_i) xi_i <xi_i, in>: g5 eps for the operator, eps g5 for the adjoint
        for (size_t k = 0; k < c.size(); ++k) z[k] = alpha * O.b * (O.D.lam[k / S.nvec] > 0 ? 1.0 : -1.0) * c[k];
        WL_TRY(defl_axpy(S, O.D, prec, out, z, !dagger, s));
        if (red_dst) {
            WL_TRY(blas(S, BL_NORM2, prec, &out[0], 1, nullptr, red_spec(S, RED_STORE, red_dst), s));
            WL_TRY(blas(S, BL_NORM2, prec, &out[1], 1, nullptr, red_spec(S, RED_ACCUM, red_dst), s));
        }
    }
    return WL_OK;
}

wl_status fetch(ExecSet &S, const double *d, std::vector<double> &h, hipStream_t s)
{
    h.resize(S.nvec);
    WL_HIP(hipMemcpyAsync(h.data(), d, sizeof(double) * S.nvec, hipMemcpyDeviceToHost, s));
    WL_HIP(hipStreamSynchronize(s));
    return WL_OK;
}

wl_status put(ExecSet &S, double *d, const std::vector<double> &h, hipStream_t s)
{
    WL_HIP(hipMemcpyAsync(d, h.data(), sizeof(double) * S.nvec, hipMemcpyHostToDevice, s));
    WL_HIP(hipStreamSynchronize(s));
    return WL_OK;
}

wl_status set_active(ExecSet &S, const std::vector<int32_t> &act, hipStream_t s)
{
    S.h_active = act;
    return S.upload_active(s);
}

wl_status common_checks(wl_gauge U, int32_t nrhs, double rho, double mass, int32_t degree, double lo, double hi,
                        double scale, int prec, int32_t recon)
{
    WL_TRY(check_gauge(U));
    if (nrhs < 1) return set_error(WL_ERR_ARG, "nrhs must be >= 1");
    if (!(rho > 0 && rho < 4)) return set_error(WL_ERR_ARG, "rho must be in (0, 4)");
    if (!(mass >= 0 && mass < 2 * rho)) return set_error(WL_ERR_ARG, "mass must be in [0, 2 rho)");
    if (degree < 1 || degree > 100000) return set_error(WL_ERR_ARG, "degree must be in [1, 100000]");
    if (!(lo > 0 && lo < hi) || !std::isfinite(hi)) return set_error(WL_ERR_ARG, "0 < lo < hi required");
    if (!std::isfinite(scale)) return set_error(WL_ERR_ARG, "scale must be finite");
    if (prec != WL_F64 && prec != WL_F32) return set_error(WL_ERR_PREC, "overlap operator runs in FP64 or FP32");
    if (!prec_recon_ok(prec, recon) || !prec_recon_ok(WL_F64, recon))
        return set_error(WL_ERR_PREC, "unsupported precision %d / recon %d", prec, recon);
    return WL_OK;
}

wl_status no_overlap(const double *a, const double *b, wl_gauge U, int nrhs)
{
    const size_t bytes = (size_t)nrhs * 2 * U->geom.Vh * 24 * sizeof(double);
    if ((const char *)a < (const char *)b + bytes && (const char *)b < (const char *)a + bytes)
        return set_error(WL_ERR_ARG, "input and output overlap");
    return WL_OK;
}

wl_status setup(wl_gauge U, int nrhs, double rho, double mass, int degree, double lo, double hi, double scale,
                int recon, const double *v0, int nev, const double *evecs, const double *evals, hipStream_t s,
                Overlap *O)
{
    if (nev < 0 || nev > 64) return set_error(WL_ERR_ARG, "nev must be in [0, 64]");
    if (nev > 0 && !evals) return set_error(WL_ERR_ARG, "null eigenvalues");
    if (nev > 0) WL_TRY(check_field(evecs, U, nev, "evecs"));
    if (!(scale > 0)) WL_TRY(hw2_scale(U, rho, v0, s, &scale));
    WL_TRY(defl_load(U, 1.0 / (8.0 - 2.0 * rho), nev, evecs, evals, s, &O->D));
    WL_TRY(get_set({SysEntry{U, nrhs, 1.0 / (8.0 - 2.0 * rho)}}, &O->S));
    std::fill(O->S->h_active.begin(), O->S->h_active.end(), 1);
    WL_TRY(O->S->upload_active(s));
    WL_TRY(sign_plan(*O->S, rho, degree, lo, hi, scale, &O->P));
    O->recon = recon;
    O->a = rho + 0.5 * mass;
    O->b = rho - 0.5 * mass;
    return WL_OK;
}

}  // namespace
}  // namespace wl

using namespace wl;

extern "C" {

wl_status overlap_dslash(wl_gauge U, const double *in, double *out, int32_t nrhs, double rho, double mass,
                         int32_t degree, double lo, double hi, double scale, int32_t dagger, wl_prec prec,
                         int32_t recon, int32_t nev, const double *evecs, const double *evals, void *stream)
{
    clear_error();
    WL_TRY(common_checks(U, nrhs, rho, mass, degree, lo, hi, scale, prec, recon));
    WL_TRY(check_field(in, U, nrhs, "in"));
    WL_TRY(check_field(out, U, nrhs, "out"));
    WL_TRY(no_overlap(in, out, U, nrhs));
    hipStream_t s = (hipStream_t)stream;
    Overlap O;
    WL_TRY(setup(U, nrhs, rho, mass, degree, lo, hi, scale, recon, in, nev, evecs, evals, s, &O));
    ExecSet &S = *O.S;
    const double *cin[1] = {in};
    double *cout[1] = {out};
    Field v[2], w[2];
    for (int p = 0; p < 2; ++p) {
        WL_TRY(S.field("ov_v" + std::to_string(p), prec, &v[p]));
        WL_TRY(S.field("ov_w" + std::to_string(p), prec, &w[p]));
        WL_TRY(pack(S, cin, p, v[p], s));
    }
    WL_TRY(ov_apply(O, prec, dagger != 0, w, v, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, s));
    for (int p = 0; p < 2; ++p) WL_TRY(unpack(S, cout, p, w[p], s));
    WL_HIP(hipStreamSynchronize(s));
    return WL_OK;
}

wl_status overlap_cg(wl_gauge U, const double *eta, double *x, int32_t nrhs, double rho, double mass,
                     int32_t degree, double lo, double hi, double scale, double tol, int32_t maxiter,
                     wl_prec sloppy, int32_t recon, double delta, int32_t nev, const double *evecs,
                     const double *evals, wl_solve_info *info, void *stream)
{
    clear_error();
    const auto t0 = std::chrono::steady_clock::now();
    WL_TRY(common_checks(U, nrhs, rho, mass, degree, lo, hi, scale, sloppy, recon));
    if (!(tol > 0) || !(tol < 1)) return set_error(WL_ERR_ARG, "tol must be in (0, 1)");
    if (maxiter < 1) return set_error(WL_ERR_ARG, "maxiter must be >= 1");
    if (!(delta > 0 && delta < 1)) return set_error(WL_ERR_ARG, "delta must be in (0, 1)");
    if (!info) return set_error(WL_ERR_ARG, "null info");
    if (!(mass > 0)) return set_error(WL_ERR_ARG, "the solve needs mass > 0 (D_ov(0) has exact zero modes)");
    WL_TRY(check_field(eta, U, nrhs, "eta"));
    WL_TRY(check_field(x, U, nrhs, "x"));
    WL_TRY(no_overlap(eta, x, U, nrhs));
    hipStream_t s = (hipStream_t)stream;
    Overlap O;
    WL_TRY(setup(U, nrhs, rho, mass, degree, lo, hi, scale, recon, eta, nev, evecs, evals, s, &O));
    ExecSet &S = *O.S;
    const int nv = S.nvec;
    const int P = sloppy;
    g_bytes_acc = 0.0;

    // FP64: eta, x, residual; working precision: correction e, tracked residual
    // rt, search direction p, q = D p, s = D^dagger rt
    Field E[2], X[2], R[2], e[2], rt[2], pp[2], q[2], sv[2];
    const double *ceta[1] = {eta};
    double *cx[1] = {x};
    for (int p = 0; p < 2; ++p) {
        const std::string t = std::to_string(p);
        WL_TRY(S.field("oc_eta" + t, P_F64, &E[p]));
        WL_TRY(S.field("oc_x" + t, P_F64, &X[p]));
        WL_TRY(S.field("oc_r" + t, P_F64, &R[p]));
        WL_TRY(S.field("oc_e" + t, P, &e[p]));
        WL_TRY(S.field("oc_rt" + t, P, &rt[p]));
        WL_TRY(S.field("oc_p" + t, P, &pp[p]));
        WL_TRY(S.field("oc_q" + t, P, &q[p]));
        WL_TRY(S.field("oc_s" + t, P, &sv[p]));
        WL_TRY(pack(S, ceta, p, E[p], s));
        WL_TRY(pack(S, cx, p, X[p], s));
    }
    double *d_rr = S.scal(SC_RR), *d_qq = S.scal(SC_QQ), *d_gg = S.scal(SC_TMP), *d_eta = S.scal(SC_ETA);
    double *d_al = S.scal(SC_ALPHA), *d_be = S.scal(SC_BETA);
    std::vector<double> eta2, rr, qq, gg, gam(nv), al(nv), be(nv);
    WL_TRY(blas(S, BL_NORM2, P_F64, &E[0], 1, nullptr, red_spec(S, RED_STORE, d_eta), s));
    WL_TRY(blas(S, BL_NORM2, P_F64, &E[1], 1, nullptr, red_spec(S, RED_ACCUM, d_eta), s));
    WL_TRY(fetch(S, d_eta, eta2, s));

    std::vector<int32_t> outer(nv, 1), inner(nv, 0);
    std::vector<double> target(nv, 0.0), resid(nv, 0.0);
    std::vector<int> iters(nv, 0), cycles(nv, 0);
    for (int v = 0; v < nv; ++v) {
        if (!std::isfinite(eta2[v])) return set_error(WL_ERR_NONFINITE, "non-finite source");
        if (eta2[v] == 0.0) outer[v] = 0;  // zero source: x = 0
    }
    for (int v = 0; v < nv; ++v)
        if (!outer[v]) {
            std::vector<int32_t> one(nv, 0);
            one[v] = 1;
            WL_TRY(set_active(S, one, s));
            for (int p = 0; p < 2; ++p) WL_TRY(blas(S, BL_ZERO, P_F64, &X[p], 1, nullptr, no_red(), s));
        }

    int total = 0;
    bool nonfinite = false;
    const int max_cycles = 100;
    for (int cyc = 0; cyc <= max_cycles; ++cyc) {
        if (std::none_of(outer.begin(), outer.end(), [](int32_t a) { return a != 0; })) break;
        WL_TRY(set_active(S, outer, s));
        // R = eta - D X in FP64, |R|^2
        WL_TRY(ov_apply(O, P_F64, false, R, X, -1.0, E, 1.0, nullptr, 0.0, d_rr, s));
        WL_TRY(fetch(S, d_rr, rr, s));
        bool any = false;
        for (int v = 0; v < nv; ++v) {
            if (!outer[v]) continue;
            if (!std::isfinite(rr[v])) {
                nonfinite = true;
                outer[v] = 0;
                continue;
            }
            resid[v] = std::sqrt(rr[v] / eta2[v]);
            if (resid[v] <= tol || total >= maxiter || cyc == max_cycles) {
                outer[v] = 0;
                continue;
            }
            // inner goal: reduce |R| by delta, but never below what the tolerance needs
            const double want = 0.5 * tol * std::sqrt(eta2[v]);
            target[v] = P == P_F64 ? want : std::max(want, delta * std::sqrt(rr[v]));
            ++cycles[v];
            any = true;
        }
        if (!any) break;
        WL_TRY(set_active(S, outer, s));
        inner = outer;
        // rt = R (working precision), e = 0, s = D^dagger rt, p = s, gam = |s|^2
        for (int p = 0; p < 2; ++p) {
            WL_TRY(convert(S, rt[p], R[p], s));
            WL_TRY(blas(S, BL_ZERO, P, &e[p], 1, nullptr, no_red(), s));
        }
        WL_TRY(ov_apply(O, P, true, sv, rt, 1.0, nullptr, 0.0, nullptr, 0.0, d_gg, s));
        WL_TRY(fetch(S, d_gg, gg, s));
        for (int v = 0; v < nv; ++v) gam[v] = gg[v];
        for (int p = 0; p < 2; ++p) {
            const Field f[2] = {pp[p], sv[p]};
            WL_TRY(blas(S, BL_COPY, P, f, 2, nullptr, no_red(), s));
        }
        while (total < maxiter) {
            // q = D p, alpha = gam / |q|^2
            WL_TRY(ov_apply(O, P, false, q, pp, 1.0, nullptr, 0.0, nullptr, 0.0, d_qq, s));
            WL_TRY(fetch(S, d_qq, qq, s));
            for (int v = 0; v < nv; ++v) al[v] = inner[v] && qq[v] > 0 ? gam[v] / qq[v] : 0.0;
            WL_TRY(put(S, d_al, al, s));
            // e += alpha p; rt -= alpha q; |rt|^2
            for (int p = 0; p < 2; ++p) {
                const Field f[4] = {e[p], pp[p], rt[p], q[p]};
                WL_TRY(blas(S, BL_CG_UPDATE, P, f, 4, d_al, red_spec(S, p == 0 ? RED_STORE : RED_ACCUM, d_rr), s));
            }
            WL_TRY(fetch(S, d_rr, rr, s));
            ++total;
            bool left = false;
            for (int v = 0; v < nv; ++v) {
                if (!inner[v]) continue;
                ++iters[v];
                if (!std::isfinite(rr[v]) || !std::isfinite(qq[v])) {
                    nonfinite = true;
                    inner[v] = outer[v] = 0;
                    continue;
                }
                if (std::sqrt(rr[v]) <= target[v]) inner[v] = 0;
                else left = true;
            }
            if (!left) break;
            WL_TRY(set_active(S, inner, s));
            // s = D^dagger rt, beta = |s|^2 / gam, p = s + beta p
            WL_TRY(ov_apply(O, P, true, sv, rt, 1.0, nullptr, 0.0, nullptr, 0.0, d_gg, s));
            WL_TRY(fetch(S, d_gg, gg, s));
            for (int v = 0; v < nv; ++v) {
                be[v] = inner[v] && gam[v] > 0 ? gg[v] / gam[v] : 0.0;
                if (inner[v]) gam[v] = gg[v];
            }
            WL_TRY(put(S, d_be, be, s));
            for (int p = 0; p < 2; ++p) {
                const Field f[2] = {pp[p], sv[p]};
                WL_TRY(blas(S, BL_XPAY, P, f, 2, d_be, no_red(), s));
            }
        }
        // X += e for every vector of this cycle
        WL_TRY(set_active(S, outer, s));
        for (int p = 0; p < 2; ++p) {
            const Field f[2] = {X[p], e[p]};
            WL_TRY(blas(S, BL_ACCUM, P, f, 2, nullptr, no_red(), s));
        }
    }
    std::vector<int32_t> all(nv, 1);
    WL_TRY(set_active(S, all, s));
    for (int p = 0; p < 2; ++p) WL_TRY(unpack(S, cx, p, X[p], s));
    WL_HIP(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool ok = true;
    for (int v = 0; v < nv; ++v) {
        wl_solve_info &I = info[v];
        I.iters = iters[v];
        I.reliable_updates = std::max(0, cycles[v] - 1);
        I.precision_escalations = 0;
        I.true_resid = eta2[v] == 0.0 ? 0.0 : resid[v];
        I.converged = eta2[v] == 0.0 || resid[v] <= tol;
        I.seconds = secs;
        I.gbytes = g_bytes_acc * 1e-9;
        ok = ok && I.converged;
    }
    if (nonfinite) return set_error(WL_ERR_NONFINITE, "non-finite value in the overlap solve");
    if (!ok) return set_error(WL_ERR_NOCONV, "overlap CG did not reach tol %g in %d iterations", tol, maxiter);
    return WL_OK;
}

}  // extern "C"
