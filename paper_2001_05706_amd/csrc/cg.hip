// cg.hip -- even-odd preconditioned Krylov solvers for the Wilson and
// Wilson-clover operators, mixed precision with FP64 reliable updates, for one
// set of systems x right-hand sides at once (QUDA_DIRAC_WILSON and
// QUDA_DIRAC_CLOVER of Table 1; the mixed-precision inverters of the QUDA line
// of work cited in Section 1): CG on the normal equations (CGNR) and BiCGStab
// on the Schur system itself.  With a clover term A the Schur operator is the
// asymmetric M = A_ee - kappa^2 D_eo A_oo^{-1} D_oe (both clover factors sit at
// output sites, so they ride in the hop epilogues), b' = eta_e +
// kappa D_eo A_oo^{-1} eta_o and psi_o = A_oo^{-1} (eta_o + kappa D_oe psi_e).
//
//   b' = eta_e + kappa D_eo eta_o,   M = 1 - kappa^2 D_eo D_oe,
//   M^+ = 1 - kappa^2 D_oe^+ D_eo^+ (dagger hops in the same order).
// Iteration (sloppy precision; alpha, beta, gamma stay on the device):
//   q = M p, alpha = gamma / |q|^2; r -= alpha q (|r|^2 fused);
//   s = M^+ r, gamma' = |s|^2, beta = gamma'/gamma; x += alpha p and
//   p = s + beta p in one pass over p.
// The host reads only the |r|^2 history, once per chunk of iterations.  A
// chunk is captured once as a HIP graph and replayed.  When the sloppy
// residual of a right-hand side has fallen by `delta` since its last update
// (or reached the tolerance, or maxiter) the FP64 accumulator takes x_lo and
// the residual b' - M x is recomputed in FP64 (reliable update); p is kept
// and s, gamma are recomputed from the new residual.  Two updates in a row
// that fail to halve the FP64 residual raise the sloppy precision one step.
// Finally psi_o = eta_o + kappa D_oe psi_e and the true residual
// |eta - D psi| / |eta| is computed in FP64 with the whole-lattice operator.
//
// BiCGStab (van der Vorst) on M x = b' with shadow residual rhat = r_0:
//   beta = (rho / rho_prev)(alpha / omega); p = r + beta (p - omega v);
//   v = M p, alpha = rho / <rhat, v>; s = r - alpha v; t = M s,
//   omega = <t, s> / |t|^2; x += alpha p + omega s; r = s - omega t;
//   rho_prev = rho, rho = <rhat, r>.
// <rhat, v> and (<t, s>, |t|^2) are reduced in the epilogue of the second hop of
// M; <rhat, r> and |r|^2 in the x/r update.  A reliable update replaces r and
// recomputes rho; a breakdown (zero <rhat, v> or |t|) or a non-finite value
// restarts from the FP64 accumulator with rhat = r.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "wl_host.h"

namespace wl {

static hipStream_t capture_stream()
{
    static hipStream_t cs = nullptr;
    if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        cs = nullptr;
    }
    return cs;
}

enum { M_CGNR = 0, M_BICGSTAB = 1 };

struct Cg {
    ExecSet &S;
    hipStream_t s;
    int method = M_CGNR;
    int recon;
    double tol;
    int maxiter;
    double delta;
    int sloppy;
    bool use_graphs;

    Field eta_e, eta_o, bp, xh, rh, t64, xo;  // FP64
    Field xl, rl, p, q, sv, tl;               // sloppy; BiCGStab: q = v, sv = s
    Field tb, rhat;                           // sloppy, BiCGStab only: t, shadow residual
    const double *c_plain = nullptr, *c_bp = nullptr, *c_M = nullptr, *c_res = nullptr, *c_tres = nullptr;

    Cg(ExecSet &S_, hipStream_t s_) : S(S_), s(s_) {}

    wl_status sloppy_fields()
    {
        WL_TRY(S.field("cg_xl", sloppy, &xl));
        WL_TRY(S.field("cg_rl", sloppy, &rl));
        WL_TRY(S.field("cg_p", sloppy, &p));
        WL_TRY(S.field("cg_q", sloppy, &q));
        WL_TRY(S.field("cg_s", sloppy, &sv));
        WL_TRY(S.field("cg_t", sloppy, &tl));
        if (method == M_BICGSTAB) {
            WL_TRY(S.field("bi_t", sloppy, &tb));
            WL_TRY(S.field("bi_rhat", sloppy, &rhat));
        }
        return WL_OK;
    }

    wl_status setup()
    {
        WL_TRY(S.field("cg_eta_e", P_F64, &eta_e));
        WL_TRY(S.field("cg_eta_o", P_F64, &eta_o));
        WL_TRY(S.field("cg_bp", P_F64, &bp));
        WL_TRY(S.field("cg_xh", P_F64, &xh));
        WL_TRY(S.field("cg_rh", P_F64, &rh));
        WL_TRY(S.field("cg_t64", P_F64, &t64));
        WL_TRY(S.field("cg_xo", P_F64, &xo));
        WL_TRY(sloppy_fields());
        std::vector<double> cp, cb, cm, cr, ct;
        for (auto &e : S.systems) {
            const double k = e.kappa;
            cp.insert(cp.end(), {0, 0, 0, 0, 1.0});
            cb.insert(cb.end(), {1.0, 0, 0, 0, k});
            cm.insert(cm.end(), {1.0, 0, 0, 0, -k * k});
            cr.insert(cr.end(), {-1.0, 1.0, 0, 0, k * k});
            ct.insert(ct.end(), {-1.0, 1.0, 0, 0, k});
        }
        WL_TRY(coef_table(S, cp, &c_plain));
        WL_TRY(coef_table(S, cb, &c_bp));
        WL_TRY(coef_table(S, cm, &c_M));
        WL_TRY(coef_table(S, cr, &c_res));
        WL_TRY(coef_table(S, ct, &c_tres));
        return WL_OK;
    }

    Epi epi(const double *coef, int nx = 0, Field x0 = Field(), Field x1 = Field(), int clov = 0)
    {
        Epi e;
        e.coef = coef;
        e.nx = nx;
        e.X[0] = x0;
        e.X[1] = x1;
        e.clov = clov;
        return e;
    }
    // the two hops of the Schur operator: t_o = A_oo^{-1} D_oe in, out = A_ee in - kappa^2 D_eo t_o
    // (A = 1 for systems without a clover term)
    Epi first(const double *coef) { return epi(coef, 0, Field(), Field(), EPI_CLOV_INV); }
    Epi second(const double *coef, int nx, Field x0, Field x1 = Field()) { return epi(coef, nx, x0, x1, EPI_CLOV_X0); }

    // out = M in (dag = false) or M^+ in (dag = true); tmp is an odd-parity field
    wl_status apply_M(int prec, int rc, bool dag, const Field &out, const Field &in, const Field &tmp,
                      const RedSpec &red, bool use_active = true)
    {
        WL_TRY(hop(S, prec, rc, dag, 1, tmp, in, first(c_plain), no_red(), s, use_active));
        WL_TRY(hop(S, prec, rc, dag, 0, out, tmp, second(c_M, 1, in), red, s, use_active));
        return WL_OK;
    }

    // rh = b' - M xh in FP64 with |rh|^2 into SC_RR.  Links are rebuilt from 12
    // reals when the caller chose recon-12 (exact to rounding for SU(3)); the
    // final true residual always uses all 18.
    wl_status residual64(bool use_active = true)
    {
        WL_TRY(hop(S, P_F64, recon, false, 1, t64, xh, first(c_plain), no_red(), s, use_active));
        WL_TRY(hop(S, P_F64, recon, false, 0, rh, t64, second(c_res, 2, xh, bp),
                   red_spec(S, RED_STORE, S.scal(SC_RR)), s, use_active));
        return WL_OK;
    }

    // iteration j of a chunk in the sloppy precision; history row j receives |r|^2
    // (CGNR: its block partials are summed for the whole chunk by hist_finalize)
    wl_status iteration(int j)
    {
        double *hist_row = S.hist + (size_t)j * S.nvec;
        if (method == M_BICGSTAB) {
            // p = r + beta (p - omega v);  v = M p, alpha = rho / <rhat, v>;  s = r - alpha v;
            // t = M s, omega = <t, s> / |t|^2;  x += alpha p + omega s;  r = s - omega t, rho = <rhat, r>
            Field fp[3] = {p, rl, q};
            WL_TRY(blas(S, BL_BICG_P, sloppy, fp, 3, nullptr, no_red(), s));
            WL_TRY(hop(S, sloppy, recon, false, 1, tl, p, first(c_plain), no_red(), s));
            WL_TRY(hop(S, sloppy, recon, false, 0, q, tl, second(c_M, 2, p, rhat),
                       red_spec(S, RED_BICG_ALPHA, nullptr, 2, RM_DOT_X1), s));
            Field fs[3] = {sv, rl, q};
            WL_TRY(blas(S, BL_BICG_S, sloppy, fs, 3, nullptr, no_red(), s));
            WL_TRY(hop(S, sloppy, recon, false, 1, tl, sv, first(c_plain), no_red(), s));
            WL_TRY(hop(S, sloppy, recon, false, 0, tb, tl, second(c_M, 1, sv),
                       red_spec(S, RED_BICG_OMEGA, nullptr, 3, RM_OUT_X0), s));
            Field fx[6] = {xl, p, sv, rl, tb, rhat};
            WL_TRY(blas(S, BL_BICG_XR, sloppy, fx, 6, nullptr, red_spec(S, RED_BICG_RHO, hist_row, 3), s));
            return WL_OK;
        }
        // q = M p, alpha = gamma / |q|^2;  r -= alpha q;  s = M^dagger r, beta;
        // then x += alpha p and p = s + beta p in one pass over p
        WL_TRY(apply_M(sloppy, recon, false, q, p, tl, red_spec(S, RED_ALPHA, nullptr)));
        Field f[2] = {rl, q};
        RedSpec rr = red_spec(S, RED_STORE, hist_row);
        rr.partials = S.hist_partials + (size_t)j * S.max_pslots;
        rr.defer = 1;
        WL_TRY(blas(S, BL_R_UPDATE, sloppy, f, 2, S.scal(SC_ALPHA), rr, s));
        WL_TRY(apply_M(sloppy, recon, true, sv, rl, tl, red_spec(S, RED_BETA, nullptr)));
        Field g[3] = {p, sv, xl};
        WL_TRY(blas(S, BL_XPAY_X, sloppy, g, 3, S.scal(SC_BETA), no_red(), s));
        return WL_OK;
    }

    double iteration_bytes()
    {
        if (method == M_BICGSTAB)  // 4 hops (+3 epilogue reads), p (4), s (3), x/r (7)
            return 4 * hop_bytes(S, sloppy, recon, true) + blas_bytes(S, sloppy, 3 + 4 + 3 + 7, true);
        return 4 * hop_bytes(S, sloppy, recon, true) + 2 * blas_bytes(S, sloppy, 1, true) +
               blas_bytes(S, sloppy, 3, true) + blas_bytes(S, sloppy, 5, true);
    }

    // The part of a refresh common to continued and restarted vectors, for the
    // vectors of the current mask: r = rh in the sloppy precision; CGNR also
    // s = M^+ r, gamma = |s|^2
    wl_status refresh_s()
    {
        WL_TRY(convert(S, rl, rh, s));
        if (method != M_CGNR) return WL_OK;
        return apply_M(sloppy, recon, true, sv, rl, tl, red_spec(S, RED_GAMMA, nullptr));
    }

    // After the FP64 residual rh is fresh: continue (cont) or restart (restart)
    // the sloppy recurrence of the active vectors.  Masks are host vectors.
    // pre: refresh_s() already ran for a superset of these vectors in the
    // current sloppy precision.
    wl_status refresh(const std::vector<int> &cont, const std::vector<int> &restart, bool pre = false)
    {
        const int nv = S.nvec;
        std::vector<int> both(nv);
        bool anyc = false, anyr = false;
        for (int v = 0; v < nv; ++v) {
            both[v] = cont[v] || restart[v];
            anyc = anyc || cont[v];
            anyr = anyr || restart[v];
        }
        if (!anyc && !anyr) return WL_OK;
        if (method == M_CGNR) {
            if (!pre) {
                S.h_active.assign(both.begin(), both.end());
                WL_TRY(S.upload_active(s));
                WL_TRY(refresh_s());
            }
            if (anyr) {  // p = s: a fresh search direction
                S.h_active.assign(restart.begin(), restart.end());
                WL_TRY(S.upload_active(s));
                Field cp[2] = {p, sv};
                WL_TRY(blas(S, BL_COPY, sloppy, cp, 2, nullptr, no_red(), s));
            }
            return WL_OK;
        }
        if (!pre) {
            S.h_active.assign(both.begin(), both.end());
            WL_TRY(S.upload_active(s));
            WL_TRY(refresh_s());
        }
        if (anyc) {  // keep rhat, p, v, alpha, omega, rho_prev; rho = <rhat, r>
            S.h_active.assign(cont.begin(), cont.end());
            WL_TRY(S.upload_active(s));
            Field cd[2] = {rhat, rl};
            WL_TRY(blas(S, BL_CDOT, sloppy, cd, 2, nullptr, red_spec(S, RED_CDOT_RHO, nullptr, 2), s));
        }
        if (anyr) {  // new shadow residual rhat = r, p = v = 0, rho = rho_prev = |r|^2, alpha = omega = 1
            S.h_active.assign(restart.begin(), restart.end());
            WL_TRY(S.upload_active(s));
            Field cp[2] = {rhat, rl};
            WL_TRY(blas(S, BL_COPY, sloppy, cp, 2, nullptr, no_red(), s));
            WL_TRY(blas(S, BL_ZERO, sloppy, &p, 1, nullptr, no_red(), s));
            WL_TRY(blas(S, BL_ZERO, sloppy, &q, 1, nullptr, no_red(), s));
            Field cd[2] = {rhat, rl};
            WL_TRY(blas(S, BL_CDOT, sloppy, cd, 2, nullptr, red_spec(S, RED_BICG_INIT, nullptr, 2), s));
        }
        return WL_OK;
    }

    wl_status chunk(int k)
    {
        if (!use_graphs || prof().on) {
            for (int j = 0; j < k; ++j) WL_TRY(iteration(j));
            if (method == M_CGNR) WL_TRY(hist_finalize(S, k, s));
            return WL_OK;
        }
        // the coefficient tables are cached by content, so their addresses name
        // the systems' kappas: a chunk captured for other kappas is not reused
        char coefs[64];
        snprintf(coefs, sizeof(coefs), "/%p/%p", (const void *)c_plain, (const void *)c_M);
        const std::string key = "cg/" + std::to_string(method) + "/" + std::to_string(k) + "/" +
                                std::to_string(sloppy) + "/" + std::to_string(recon) + coefs;
        auto it = S.graphs.find(key);
        if (it == S.graphs.end()) {
            const SysDesc *tab = nullptr;  // packed links and tables exist before capture
            WL_TRY(S.sys_table(sloppy, recon, s, &tab));
            hipStream_t cs = capture_stream();
            if (!cs) return set_error(WL_ERR_HIP, "cannot create the capture stream");
            const double saved = g_bytes_acc;
            hipStream_t user = s;
            s = cs;
            WL_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
            wl_status st = WL_OK;
            for (int j = 0; j < k && st == WL_OK; ++j) st = iteration(j);
            if (st == WL_OK && method == M_CGNR) st = hist_finalize(S, k, s);
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(cs, &g);
            s = user;
            g_bytes_acc = saved;
            if (st != WL_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (ce != hipSuccess) return set_error(WL_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ce));
            hipGraphExec_t ex = nullptr;
            hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) return set_error(WL_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
            it = S.graphs.emplace(key, ex).first;
        }
        g_bytes_acc += k * iteration_bytes();
        WL_HIP(hipGraphLaunch(it->second, s));
        return WL_OK;
    }
};

// Waits for event e by polling it: the readbacks inside the solve loop are a
// few hundred bytes that the host needs at once, and a blocking wait adds the
// thread's wake-up to every one of them.  After the first few thousand polls
// the thread yields between polls, and a wait longer than WL_WAIT_TIMEOUT_S
// seconds (default 600) returns an error instead of spinning on a GPU that
// no longer answers.
static wl_status wait_spin(hipEvent_t e)
{
    static const double limit = [] {
        const char *v = getenv("WL_WAIT_TIMEOUT_S");
        const double t = v ? atof(v) : 0.0;
        return t > 0.0 ? t : 600.0;
    }();
    const auto t0 = std::chrono::steady_clock::now();
    for (long n = 0;; ++n) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipSuccess) return WL_OK;
        if (q != hipErrorNotReady) return set_error(WL_ERR_HIP, "waiting for a readback: %s", hipGetErrorString(q));
        if (n >= 4096) {
            std::this_thread::yield();
            if ((n & 1023) == 0 &&
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit)
                return set_error(WL_ERR_HIP, "a readback did not complete within %.0f s", limit);
        }
    }
}

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static int round_chunk(double k)
{
    static const int sizes[] = {2, 3, 4, 6, 8, 12, 16, 24, 32};
    int best = sizes[0];
    for (int c : sizes)
        if (c <= k) best = c;
    return best;
}

// Solve the systems of S for the canonical sources eta[i] into x[i] (guesses on entry).
wl_status run_cg(ExecSet &S, const double *const *eta, double *const *x, int recon, double tol, int maxiter,
                 int sloppy, double delta, wl_solve_info *info, hipStream_t s, int method = M_CGNR)
{
    const double t0 = now_s();
    g_bytes_acc = 0.0;
    Cg cg(S, s);
    cg.method = method;
    cg.recon = recon;
    cg.tol = tol;
    cg.maxiter = maxiter;
    cg.delta = delta;
    cg.sloppy = sloppy;
    const char *ge = getenv("WL_GRAPHS");
    cg.use_graphs = !(ge && ge[0] == '0');
    const bool trace = getenv("WL_DEBUG") != nullptr;  // per-chunk solver trace on stderr
    WL_TRY(cg.setup());
    const int nv = S.nvec;
    double *hp = S.h_pinned;  // [kHist * nv] history, then scalars

    std::fill(S.h_active.begin(), S.h_active.end(), 1);
    WL_TRY(S.upload_active(s));
    WL_HIP(hipMemsetAsync(S.bad, 0, sizeof(int32_t) * nv, s));

    // sources, |eta|^2, b', initial guess, first FP64 residual
    WL_TRY(pack(S, eta, 0, cg.eta_e, s));
    WL_TRY(pack(S, eta, 1, cg.eta_o, s));
    WL_TRY(blas(S, BL_NORM2, P_F64, &cg.eta_e, 1, nullptr, red_spec(S, RED_STORE, S.scal(SC_ETA)), s));
    WL_TRY(blas(S, BL_NORM2, P_F64, &cg.eta_o, 1, nullptr, red_spec(S, RED_ACCUM, S.scal(SC_ETA)), s));
    // b' = eta_e + kappa D_eo A_oo^{-1} eta_o (xo holds A_oo^{-1} eta_o until psi_o is formed)
    Field src_o = cg.eta_o;
    if (S.has_clover) {
        const Field f[2] = {cg.xo, cg.eta_o};
        WL_TRY(blas(S, BL_CLOV_INV, P_F64, f, 2, nullptr, no_red(), s, true, 1));
        src_o = cg.xo;
    }
    // (|b'|^2 rides on that hop: it is |r|^2 for a zero initial guess)
    WL_TRY(hop(S, P_F64, 18, false, 0, cg.bp, src_o, cg.epi(cg.c_bp, 1, cg.eta_e),
               red_spec(S, RED_STORE, S.scal(SC_RR)), s));
    WL_TRY(pack(S, (const double *const *)x, 0, cg.xh, s));
    // r = b' - M x.  When every initial guess is zero (the usual start) r = b'
    // exactly and the residual's two FP64 hops are replaced by a copy: the
    // guesses' |x_e|^2 are read back first to decide.
    WL_TRY(blas(S, BL_NORM2, P_F64, &cg.xh, 1, nullptr, red_spec(S, RED_STORE, S.scal(SC_TMP)), s));
    WL_HIP(hipMemcpyAsync(hp, S.scal(SC_TMP), sizeof(double) * nv, hipMemcpyDeviceToHost, s));
    WL_HIP(hipStreamSynchronize(s));
    bool zero_guess = true;
    for (int v = 0; v < nv; ++v) zero_guess = zero_guess && hp[v] == 0.0;
    if (zero_guess)
        WL_TRY(convert(S, cg.rh, cg.bp, s));
    else
        WL_TRY(cg.residual64());
    WL_HIP(hipMemcpyAsync(hp, S.sc, sizeof(double) * ExecSet::SC_N * nv, hipMemcpyDeviceToHost, s));
    WL_HIP(hipStreamSynchronize(s));
    std::vector<double> eta_n(nv), rmax(nv), last_true(nv), target(nv);
    std::vector<int> iters(nv, 0), updates(nv, 0), conv(nv, 0), done(nv, 0), stall(nv, 0);
    std::vector<int> zero_src(nv, 0);
    for (int v = 0; v < nv; ++v) {
        eta_n[v] = std::sqrt(hp[SC_ETA * nv + v]);
        const double r = std::sqrt(hp[SC_RR * nv + v]);
        target[v] = tol * eta_n[v];
        if (!std::isfinite(eta_n[v]) || !std::isfinite(r))
            return set_error(WL_ERR_NONFINITE, "non-finite source or initial guess (rhs %d)", v);
        if (eta_n[v] == 0.0) {
            zero_src[v] = 1;
            done[v] = conv[v] = 1;
        } else if (r <= target[v]) {
            done[v] = conv[v] = 1;
        }
        rmax[v] = last_true[v] = r;
    }
    // zero sources give x = 0
    bool anyzero = false;
    for (int v = 0; v < nv; ++v) {
        S.h_active[v] = zero_src[v];
        anyzero = anyzero || zero_src[v];
    }
    if (anyzero) {
        WL_TRY(S.upload_active(s));
        WL_TRY(blas(S, BL_ZERO, P_F64, &cg.xh, 1, nullptr, no_red(), s));
    }
    for (int v = 0; v < nv; ++v) S.h_active[v] = !done[v];
    WL_TRY(S.upload_active(s));
    bool any = false;
    for (int v = 0; v < nv; ++v) any = any || !done[v];
    int escalations = 0;
    wl_status status = WL_OK;

    if (any) {
        WL_TRY(blas(S, BL_ZERO, cg.sloppy, &cg.xl, 1, nullptr, no_red(), s));
        {
            std::vector<int> none(nv, 0), start(nv, 0);
            for (int v = 0; v < nv; ++v) start[v] = !done[v];
            WL_TRY(cg.refresh(none, start));
        }
        int k = 4;
        bool first = true;
        // FP16/BF16 recurrences drift faster: shorter chunks, so updates are not late
        auto kmax = [&]() { return cg.sloppy == P_F16 || cg.sloppy == P_BF16 ? 8.0 : 32.0; };
        auto kfrac = [&]() { return cg.sloppy == P_F16 || cg.sloppy == P_BF16 ? 0.6 : 1.0; };
        std::vector<double> rmin(nv);
        for (int v = 0; v < nv; ++v) rmin[v] = rmax[v];
        // iterations since the last update and length of the last full interval:
        // a recurrence that crawls far beyond its usual interval has lost its way
        std::vector<int> since(nv, 0), interval(nv, 8), crawl(nv, 0);
        std::vector<double> rsloppy(nv, 0.0);  // sloppy |r| at the end of the last chunk
        // CGNR: the fastest convergence (decades of the FP64 residual per
        // iteration) of an interval between two updates, the first interval
        // (the start-up transient) excluded, and the count of consecutive
        // chunks whose recurrence converged at under a third of it.  After an
        // update that continues the search direction, a half-precision
        // recurrence can lose conjugacy and crawl (32^3x64 FP16, delta 0.03:
        // 0.009 decades per iteration against 0.14 before, for 144 iterations
        // until the interval rule fired); two such chunks in a row count as a
        // crawl, which restarts the direction.
        std::vector<double> ref_rate(nv, 0.0);
        std::vector<int> slow(nv, 0);
        // raise the sloppy precision one step; p is converted (restarted vectors overwrite it)
        // `folded` marks the vectors whose sloppy solution is already in the FP64
        // accumulator with a fresh FP64 residual; the others are folded in here first
        auto escalate = [&](const char *why, const std::vector<int> &folded) -> wl_status {
            bool rest = false;
            for (int v = 0; v < nv; ++v) {
                S.h_active[v] = !done[v] && !folded[v];
                rest = rest || S.h_active[v];
            }
            if (rest) {
                WL_TRY(S.upload_active(s));
                Field ac[2] = {cg.xh, cg.xl};
                WL_TRY(blas(S, BL_ACCUM, cg.sloppy, ac, 2, nullptr, no_red(), s));
                WL_TRY(cg.residual64());
            }
            const int next = cg.sloppy == P_F32 ? P_F64 : P_F32;
            Field p_old = cg.p, v_old = cg.q, rhat_old = cg.rhat;
            cg.sloppy = next;
            WL_TRY(cg.sloppy_fields());
            for (int v = 0; v < nv; ++v) S.h_active[v] = !done[v];
            WL_TRY(S.upload_active(s));
            WL_TRY(convert(S, cg.p, p_old, s));
            if (cg.method == M_BICGSTAB) {
                WL_TRY(convert(S, cg.q, v_old, s));
                WL_TRY(convert(S, cg.rhat, rhat_old, s));
            }
            WL_TRY(blas(S, BL_ZERO, cg.sloppy, &cg.xl, 1, nullptr, no_red(), s));
            ++escalations;
            if (trace) fprintf(stderr, "[wl cg] %s: sloppy precision raised to %d\n", why, cg.sloppy);
            return WL_OK;
        };
        while (true) {
            // the first chunk runs eagerly: it tunes launch shapes and builds layouts before capture
            const bool graphs = cg.use_graphs;
            if (first) cg.use_graphs = false;
            WL_TRY(cg.chunk(k));
            cg.use_graphs = graphs;
            first = false;
            // the k history rows and the flags behind the whole history, in one copy
            WL_HIP(hipMemcpyAsync(hp, S.hist, sizeof(double) * ExecSet::kHist * nv + sizeof(int32_t) * nv,
                                  hipMemcpyDeviceToHost, s));
            int32_t *hbad = (int32_t *)(hp + (size_t)ExecSet::kHist * nv);
            WL_HIP(hipEventRecord(S.rr_ev, s));
            WL_TRY(wait_spin(S.rr_ev));
            if (trace) {
                double sc[ExecSet::SC_N];
                for (int j = 0; j < ExecSet::SC_N; ++j)
                    WL_HIP(hipMemcpy(&sc[j], S.scal(j), sizeof(double), hipMemcpyDeviceToHost));
                fprintf(stderr, "[wl cg] chunk k=%d prec=%d rhs0: |r| %.3e -> %.3e  alpha %.3e beta %.3e gamma %.3e bad %d\n",
                        k, cg.sloppy, std::sqrt(hp[0]), std::sqrt(hp[(size_t)(k - 1) * nv]), sc[SC_ALPHA],
                        sc[SC_BETA], sc[SC_GAM], (int)hbad[0]);
            }
            std::vector<int> upd(nv, 0), restart(nv, 0);
            bool anyupd = false, anybad = false;
            double rate = 0.0;
            int nrate = 0;
            for (int v = 0; v < nv; ++v) {
                if (done[v]) continue;
                iters[v] += k;
                double rfirst = 0, rlast = 0, rlow = 1e300;
                bool bad_v = hbad[v] != 0;
                for (int j = 0; j < k; ++j) {
                    const double r = std::sqrt(hp[(size_t)j * nv + v]);
                    if (!std::isfinite(r)) {
                        bad_v = true;
                        break;
                    }
                    if (j == 0) rfirst = r;
                    rlast = r;
                    rsloppy[v] = r;
                    rlow = std::min(rlow, r);
                    if (r <= target[v] || r < delta * rmax[v]) upd[v] = 1;
                }
                if (bad_v) {
                    // the sloppy state is lost: restart from the FP64 accumulator
                    upd[v] = restart[v] = 1;
                    anybad = true;
                } else {
                    if (rlow >= rmin[v]) upd[v] = 1;  // no progress over a whole chunk
                    rmin[v] = std::min(rmin[v], rlow);
                    if (rfirst > 0 && rlast > 0 && k > 1) {
                        // fastest convergence among the vectors sets the pace
                        const double cr = std::log10(rfirst / rlast) / (k - 1);
                        rate = std::max(rate, cr);
                        nrate = 1;
                        if (cg.method == M_CGNR && ref_rate[v] > 0.0)
                            slow[v] = cr < ref_rate[v] / 3 ? slow[v] + 1 : 0;
                    }
                }
                since[v] += k;
                crawl[v] = !upd[v] && (since[v] > std::max(3 * interval[v], 24) || (slow[v] >= 2 && since[v] >= 8));
                if (crawl[v]) upd[v] = 1;
                if (iters[v] >= maxiter) upd[v] = 1;
                anyupd = anyupd || upd[v];
            }
            if (anybad && cg.sloppy == P_F64) {
                status = set_error(WL_ERR_NONFINITE, "non-finite value in the FP64 iteration");
                break;
            }
            if (anyupd) {
                bool anyrst = false;
                for (int v = 0; v < nv; ++v) {
                    S.h_active[v] = upd[v] && !restart[v];
                    anyrst = anyrst || restart[v];
                }
                WL_TRY(S.upload_active(s));
                Field ac[2] = {cg.xh, cg.xl};
                WL_TRY(blas(S, BL_ACCUM, cg.sloppy, ac, 2, nullptr, no_red(), s));
                if (anyrst) {
                    for (int v = 0; v < nv; ++v) S.h_active[v] = restart[v];
                    WL_TRY(S.upload_active(s));
                    WL_TRY(blas(S, BL_ZERO, cg.sloppy, &cg.xl, 1, nullptr, no_red(), s));
                }
                for (int v = 0; v < nv; ++v) S.h_active[v] = upd[v];
                WL_TRY(S.upload_active(s));
                WL_TRY(cg.residual64());
                WL_HIP(hipMemcpyAsync(hp, S.scal(SC_RR), sizeof(double) * nv, hipMemcpyDeviceToHost, s));
                WL_HIP(hipEventRecord(S.rr_ev, s));
                // every updated vector that goes on (continued or restarted) needs
                // r from the new residual, and for CGNR s = M^+ r: they are queued
                // before the host has read it, so the GPU works while the host
                // decides (wasted only for vectors found converged)
                const double b0 = g_bytes_acc;
                WL_TRY(cg.refresh_s());
                const double spec_bytes = g_bytes_acc - b0;
                bool pre = true;
                WL_TRY(wait_spin(S.rr_ev));
                bool stalled = false;
                for (int v = 0; v < nv; ++v) {
                    if (!upd[v]) continue;
                    const double r = std::sqrt(hp[v]);
                    if (trace)
                        fprintf(stderr, "[wl cg] update rhs %d after %d iters: FP64 |r|/|eta| = %.3e (prev %.3e)%s\n", v,
                                iters[v], r / eta_n[v], last_true[v] / eta_n[v], restart[v] ? " restart" : "");
                    ++updates[v];
                    if (!std::isfinite(r)) {
                        status = set_error(WL_ERR_NONFINITE, "non-finite FP64 residual (rhs %d)", v);
                        break;
                    }
                    if (r <= target[v]) {
                        done[v] = conv[v] = 1;
                    } else if (iters[v] >= maxiter) {
                        done[v] = 1;
                    } else if (!restart[v]) {
                        // no halving of the FP64 residual, or a crawl: the search
                        // direction is stale -- restart it; a second one in a row
                        // raises the sloppy precision
                        if (r > 0.5 * last_true[v] || crawl[v]) {
                            ++stall[v];
                            restart[v] = 1;
                        } else {
                            stall[v] = 0;
                        }
                        // the recurrence drifted from the true residual: p no longer
                        // fits the new residual, so the direction restarts
                        if (rsloppy[v] > 0 && (r > 1.1 * rsloppy[v] || r < rsloppy[v] / 1.1)) restart[v] = 1;
                        if (stall[v] >= 2) stalled = true;
                    }
                    if (!crawl[v] && since[v] > 0) interval[v] = since[v];
                    if (updates[v] >= 2 && since[v] > 0 && r > 0.0 && r < last_true[v])
                        ref_rate[v] = std::max(ref_rate[v], std::log10(last_true[v] / r) / since[v]);
                    slow[v] = 0;
                    since[v] = 0;
                    last_true[v] = r;
                    rmax[v] = rmin[v] = r;
                }
                if (status != WL_OK) break;
                // after the FP64 accumulation above, so no vector loses its sloppy progress
                if ((stalled || anybad) && cg.sloppy != P_F64) {
                    WL_TRY(escalate(anybad ? "non-finite sloppy iterate" : "stagnation", upd));
                    pre = false;  // r and s are formed anew in the raised precision
                    WL_HIP(hipMemsetAsync(S.bad, 0, sizeof(int32_t) * nv, s));
                    // every vector restarts its search direction in the new precision
                    for (int v = 0; v < nv; ++v)
                        if (!done[v]) {
                            upd[v] = restart[v] = 1;
                            stall[v] = 0;
                            since[v] = 0;
                            slow[v] = 0;
                        }
                }
                std::vector<int> cont(nv, 0), rst(nv, 0);
                for (int v = 0; v < nv; ++v) {
                    cont[v] = upd[v] && !done[v] && !restart[v];
                    rst[v] = restart[v] && !done[v];
                }
                // the byte count keeps only the queued work that was used: none after
                // an escalation, else that of the vectors that go on (per-vector
                // bytes are proportional to the sites of the vector's system)
                if (spec_bytes > 0.0) {
                    double wu = 0.0, wn = 0.0;
                    for (int v = 0; v < nv; ++v) {
                        if (!upd[v]) continue;
                        const double w = (double)S.systems[S.vec[v].sys].g->geom.Vh;
                        wu += w;
                        if (!pre || !(cont[v] || rst[v])) wn += w;
                    }
                    if (wu > 0.0) g_bytes_acc -= spec_bytes * wn / wu;
                }
                WL_TRY(cg.refresh(cont, rst, pre));
            }
            bool left = false;
            for (int v = 0; v < nv; ++v) {
                S.h_active[v] = !done[v];
                left = left || !done[v];
            }
            if (!left) break;
            WL_TRY(S.upload_active(s));
            // next chunk spans about one reliable-update interval (less in half precision)
            if (nrate > 0 && rate / nrate > 1e-3) {
                const double want = kfrac() * std::log10(1.0 / delta) / (rate / nrate);
                k = round_chunk(std::min(kmax(), std::max(2.0, want)));
            } else {
                k = round_chunk(std::min(kmax(), (double)k));
            }
        }
    }

    // odd sites, true residual with the whole-lattice operator, unpack
    std::fill(S.h_active.begin(), S.h_active.end(), 1);
    WL_TRY(S.upload_active(s));
    // psi_o = A_oo^{-1} (eta_o + kappa D_oe psi_e); true residual eta - (A - kappa H) psi per parity
    WL_TRY(hop(S, P_F64, 18, false, 1, cg.xo, cg.xh, cg.epi(cg.c_bp, 1, cg.eta_o, Field(), EPI_CLOV_INV), no_red(), s));
    WL_TRY(hop(S, P_F64, 18, false, 0, cg.rh, cg.xo, cg.epi(cg.c_tres, 2, cg.xh, cg.eta_e, EPI_CLOV_X0),
               red_spec(S, RED_STORE, S.scal(SC_RR)), s));
    WL_TRY(hop(S, P_F64, 18, false, 1, cg.t64, cg.xh, cg.epi(cg.c_tres, 2, cg.xo, cg.eta_o, EPI_CLOV_X0),
               red_spec(S, RED_ACCUM, S.scal(SC_RR)), s));
    WL_TRY(unpack(S, x, 0, cg.xh, s));
    WL_TRY(unpack(S, x, 1, cg.xo, s));
    WL_HIP(hipMemcpyAsync(hp, S.scal(SC_RR), sizeof(double) * nv, hipMemcpyDeviceToHost, s));
    WL_HIP(hipStreamSynchronize(s));
    const double t1 = now_s();
    bool allconv = true;
    for (int v = 0; v < nv; ++v) {
        const double tr = eta_n[v] > 0 ? std::sqrt(hp[v]) / eta_n[v] : 0.0;
        if (info) {
            info[v].iters = iters[v];
            info[v].reliable_updates = updates[v];
            info[v].converged = conv[v] && std::isfinite(tr);
            info[v].precision_escalations = escalations;
            info[v].true_resid = tr;
            info[v].seconds = t1 - t0;
            info[v].gbytes = g_bytes_acc * 1e-9;
        }
        allconv = allconv && conv[v];
    }
    if (status != WL_OK) return status;
    if (!allconv) return set_error(WL_ERR_NOCONV, "maxiter %d reached before tol %g", maxiter, tol);
    return WL_OK;
}

}  // namespace wl

using namespace wl;

static wl_status check_solver_args(double tol, int32_t maxiter, wl_prec sloppy, int32_t recon, double delta)
{
    if (!(tol > 0) || !std::isfinite(tol)) return set_error(WL_ERR_ARG, "tol must be > 0");
    if (maxiter < 1) return set_error(WL_ERR_ARG, "maxiter must be >= 1");
    if (!(delta > 0 && delta < 1)) return set_error(WL_ERR_ARG, "delta must be in (0, 1)");
    if (!prec_recon_ok(sloppy, recon)) return set_error(WL_ERR_PREC, "unsupported sloppy precision %d / recon %d", sloppy, recon);
    return WL_OK;
}

namespace wl {
wl_status check_gauge(wl_gauge U);
wl_status check_field(const void *p, wl_gauge U, int nrhs, const char *what);
}  // namespace wl

extern "C" {

wl_status wilson_cg(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double tol,
                    int32_t maxiter, wl_prec sloppy, int32_t recon, double delta, wl_solve_info *info, void *stream)
{
    clear_error();
    WL_TRY(check_gauge(U));
    if (nrhs < 1) return set_error(WL_ERR_ARG, "nrhs = %d must be >= 1", nrhs);
    if (!(kappa > 0) || !std::isfinite(kappa)) return set_error(WL_ERR_ARG, "kappa must be > 0 and finite");
    WL_TRY(check_solver_args(tol, maxiter, sloppy, recon, delta));
    WL_TRY(check_field(eta, U, nrhs, "eta"));
    WL_TRY(check_field(x, U, nrhs, "x"));
    ExecSet *S = nullptr;
    WL_TRY(get_set({SysEntry{U, nrhs, kappa}}, &S));
    const double *e[1] = {eta};
    double *xx[1] = {x};
    return run_cg(*S, e, xx, recon, tol, maxiter, sloppy, delta, info, (hipStream_t)stream);
}

wl_status wilson_bicgstab(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double tol,
                          int32_t maxiter, wl_prec sloppy, int32_t recon, double delta, wl_solve_info *info,
                          void *stream)
{
    clear_error();
    WL_TRY(check_gauge(U));
    if (nrhs < 1) return set_error(WL_ERR_ARG, "nrhs = %d must be >= 1", nrhs);
    if (!(kappa > 0) || !std::isfinite(kappa)) return set_error(WL_ERR_ARG, "kappa must be > 0 and finite");
    WL_TRY(check_solver_args(tol, maxiter, sloppy, recon, delta));
    WL_TRY(check_field(eta, U, nrhs, "eta"));
    WL_TRY(check_field(x, U, nrhs, "x"));
    ExecSet *S = nullptr;
    WL_TRY(get_set({SysEntry{U, nrhs, kappa}}, &S));
    const double *e[1] = {eta};
    double *xx[1] = {x};
    return run_cg(*S, e, xx, recon, tol, maxiter, sloppy, delta, info, (hipStream_t)stream, M_BICGSTAB);
}

static wl_status clover_solve(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double csw,
                              double tol, int32_t maxiter, wl_prec sloppy, int32_t recon, double delta,
                              wl_solve_info *info, void *stream, int method)
{
    clear_error();
    WL_TRY(check_gauge(U));
    if (nrhs < 1) return set_error(WL_ERR_ARG, "nrhs = %d must be >= 1", nrhs);
    if (!(kappa > 0) || !std::isfinite(kappa)) return set_error(WL_ERR_ARG, "kappa must be > 0 and finite");
    if (!(csw >= 0) || !std::isfinite(csw)) return set_error(WL_ERR_ARG, "c_sw must be >= 0 and finite");
    WL_TRY(check_solver_args(tol, maxiter, sloppy, recon, delta));
    WL_TRY(check_field(eta, U, nrhs, "eta"));
    WL_TRY(check_field(x, U, nrhs, "x"));
    ExecSet *S = nullptr;
    WL_TRY(get_set({SysEntry{U, nrhs, kappa, csw}}, &S));
    const double *e[1] = {eta};
    double *xx[1] = {x};
    return run_cg(*S, e, xx, recon, tol, maxiter, sloppy, delta, info, (hipStream_t)stream, method);
}

wl_status wilson_clover_cg(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double csw,
                           double tol, int32_t maxiter, wl_prec sloppy, int32_t recon, double delta,
                           wl_solve_info *info, void *stream)
{
    return clover_solve(U, eta, x, nrhs, kappa, csw, tol, maxiter, sloppy, recon, delta, info, stream, M_CGNR);
}

wl_status wilson_clover_bicgstab(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double csw,
                                 double tol, int32_t maxiter, wl_prec sloppy, int32_t recon, double delta,
                                 wl_solve_info *info, void *stream)
{
    return clover_solve(U, eta, x, nrhs, kappa, csw, tol, maxiter, sloppy, recon, delta, info, stream, M_BICGSTAB);
}

wl_status wilson_cg_multi(int32_t nsys, const wl_gauge *U, const double *const *eta, double *const *x,
                          const int32_t *nrhs, const double *kappa, double tol, int32_t maxiter, wl_prec sloppy,
                          int32_t recon, double delta, wl_solve_info *info, void *stream)
{
    clear_error();
    if (nsys < 1 || nsys > kMaxSys) return set_error(WL_ERR_ARG, "nsys must be in [1, %d]", kMaxSys);
    if (!U || !eta || !x || !nrhs || !kappa) return set_error(WL_ERR_ARG, "null array argument");
    WL_TRY(check_solver_args(tol, maxiter, sloppy, recon, delta));
    std::vector<SysEntry> sys;
    for (int i = 0; i < nsys; ++i) {
        WL_TRY(check_gauge(U[i]));
        if (nrhs[i] < 1) return set_error(WL_ERR_ARG, "nrhs[%d] must be >= 1", i);
        if (!(kappa[i] > 0) || !std::isfinite(kappa[i])) return set_error(WL_ERR_ARG, "kappa[%d] must be > 0", i);
        WL_TRY(check_field(eta[i], U[i], nrhs[i], "eta[i]"));
        WL_TRY(check_field(x[i], U[i], nrhs[i], "x[i]"));
        sys.push_back(SysEntry{U[i], nrhs[i], kappa[i]});
    }
    ExecSet *S = nullptr;
    WL_TRY(get_set(sys, &S));
    return run_cg(*S, eta, x, recon, tol, maxiter, sloppy, delta, info, (hipStream_t)stream);
}

}  // extern "C"
