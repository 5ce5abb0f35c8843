/*
 * wilson.h -- C ABI of the MI355X (gfx950) Wilson-Dirac inverter library.
 *
 * The library applies the Wilson-Dirac D-slash (the kernel Table 2 of the paper
 * measures, with SU(3) links compressed to 12 reals as its caption states),
 * solves the Wilson system with even-odd preconditioned CG on the normal
 * equations in mixed precision (QUDA_DIRAC_WILSON, Table 1; mixed-precision
 * inverters of the QUDA line of work cited in Section 1), solves batches of
 * systems in one launch sequence, and applies the Chebyshev-polynomial sign
 * function of the Wilson kernel used by GWU-code's overlap inverter
 * (Sections 1 and 3).  The paper prints no formula; the definitions below are
 * the textbook ones.
 *
 * Canonical layouts (the only layouts a caller sees).  Complex numbers are
 * interleaved (re, im) doubles.
 *   lattice   L = (Lx, Ly, Lz, Lt), every L even and >= 2;
 *             site s = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2, even = 0
 *   links     U[s][mu][a][b]      3x3 row-major, mu = 0..3 = x, y, z, t;
 *             U_mu(x) transports the field at x+mu to x; every U must be SU(3)
 *             for the 12-real compression (recon = 12) to be exact
 *   spinors   psi[r][s][spin][col] DeGrand-Rossi gamma basis, r = RHS index
 *
 * Operators:
 *   (H psi)(x) = sum_mu b (1 - g_mu) U_mu(x) psi(x+mu) + b (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)
 *   b = -1 on hops across the time boundary when t is antiperiodic, else +1;
 *   H^+ swaps (1 - g_mu) and (1 + g_mu).  D = 1 - kappa H (kappa normalisation).
 *   Overlap kernel H_W = g5 ((4 + m0) - H/2) with m0 = -rho.
 *
 * Ownership and memory: every field pointer is a DEVICE pointer (hipMalloc'd
 * or torch-allocated) owned by the caller; the library never frees it.  The
 * library owns a wl_gauge (packed copies of the links in each precision and
 * compression asked for so far, built lazily) and its internal workspaces.
 * Handles are not thread-safe: one host thread per handle at a time.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * All device work of a call is enqueued on it.  wilson_dslash returns without
 * synchronising; solver and sign-function calls synchronise the stream before
 * they return because they fill host-side results.  Calls on one handle share
 * its packed fields and workspaces: the caller orders them, either by issuing
 * them on one stream or by making a later call's stream wait for the earlier
 * call's work (hipStreamWaitEvent); a call that returned after synchronising
 * its stream needs nothing more.  The packed copies of the links and of the
 * clover term are the exception: each is built once, on the stream of the
 * call that first needs it, and a call on another stream waits for that build
 * by itself.
 *
 * Errors: every entry point returns a wl_status and never aborts or throws.
 * Arguments are validated before any device work; wl_last_error() returns a
 * thread-local description of the most recent failure.  A pointer that
 * hipPointerGetAttributes does not report as device memory is WL_ERR_ARG.
 *
 * Environment (read at each call; none is needed for normal use):
 *   WL_TUNE=0            no autotuning: every hop runs 256-thread blocks
 *   WL_TUNE_FORCE=v:b[:c] pin the hop launches whose tuner candidates hold
 *                        variant v with block size b (column height c, 4 by
 *                        default) -- for tests of each variant
 *   WL_GRAPHS=0          solver iteration chunks launched kernel by kernel
 *                        instead of replayed from captured HIP graphs
 *   WL_STREAM_FIELDS=0|1 force the solver kernels' non-temporal field access
 *                        off or on (by default on when eight fields of the
 *                        set exceed the 256 MB last-level cache)
 *   WL_WAIT_TIMEOUT_S=n  seconds a solver waits for a device readback before
 *                        it returns WL_ERR_HIP (default 600)
 *   WL_DEBUG=1           tuner choices and a per-chunk solver trace on stderr
 * None of them changes a result beyond floating-point rounding order:
 * WL_GRAPHS and WL_STREAM_FIELDS give bit-identical solves; a launch
 * configuration can change the grouping of the reductions' partial sums.
 */
#ifndef WILSON_MI355X_H
#define WILSON_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WL_OK = 0,
    WL_ERR_ARG = 1,       /* null / non-device pointer, bad scalar argument */
    WL_ERR_GEOM = 2,      /* lattice dims not all even and >= 2, or too large */
    WL_ERR_PREC = 3,      /* unsupported precision / compression combination */
    WL_ERR_NOMEM = 4,     /* device allocation failed */
    WL_ERR_HIP = 5,       /* a HIP runtime call failed */
    WL_ERR_NOCONV = 6,    /* solver reached maxiter; x holds the last iterate */
    WL_ERR_NONFINITE = 7  /* NaN or Inf met in a reduction or an input */
} wl_status;

/* Storage precision of fields.  Arithmetic is FP64 for WL_F64 and FP32
 * otherwise; WL_F16 / WL_BF16 spinors carry one FP32 norm per site
 * (stored value = v / max|v| over the site's 24 reals). */
typedef enum { WL_F64 = 0, WL_F32 = 1, WL_F16 = 2, WL_BF16 = 3 } wl_prec;

typedef struct {
    int32_t L[4];            /* Lx, Ly, Lz, Lt: each even, >= 2 */
    int32_t antiperiodic_t;  /* 1: antiperiodic in time, 0: periodic */
} wl_geom;

typedef struct {
    int32_t iters;                 /* sloppy CG iterations */
    int32_t reliable_updates;      /* FP64 residual recomputations */
    int32_t converged;             /* 1 if true_resid <= tol */
    int32_t precision_escalations; /* sloppy precision raised after stagnation */
    double true_resid;             /* |eta - D psi| / |eta|, FP64, whole-lattice operator */
    double seconds;                /* wall time of the solve (host clock) */
    double gbytes;                 /* algorithmic HBM bytes of all kernels launched, 1e9 B */
} wl_solve_info;

typedef struct wl_gauge_s *wl_gauge;

/* ---------------------------------------------------------------- gauge */

/* Build a gauge handle from canonical FP64 links U_dev (device pointer,
 * 4 * V * 9 complex doubles).  The links are copied; U_dev may be freed after
 * the call returns.  Packed copies per precision are created lazily on first
 * use, on the stream of that call. */
wl_status wl_gauge_create(const wl_geom *geom, const double *U_dev, void *stream, wl_gauge *out);

/* Release a handle and all device memory it owns.  NULL is ignored. */
void wl_gauge_destroy(wl_gauge U);

/* ---------------------------------------------------------------- dslash */

/* The Wilson D-slash of Table 2 on nrhs canonical fields in -> out (device).
 *   parity 0 / 1: out_p = H_{p,1-p} in_{1-p} -- the single-parity hopping term
 *                 (1320 flop per output site); out is zero on the other parity
 *   parity -1   : out = D in = in - kappa H in on the whole lattice
 * dagger = 1 applies H^+ instead of H.  Arithmetic and storage follow prec
 * (in and out are converted to and from the packed layout inside the call);
 * recon = 12 (two rows, third rebuilt) or 18 (full matrix; WL_F64/WL_F32 only).
 * in and out must not overlap.  Asynchronous on `stream`. */
wl_status wilson_dslash(wl_gauge U, const double *in, double *out, int32_t nrhs, double kappa,
                        int32_t parity, int32_t dagger, wl_prec prec, int32_t recon, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * operation as wilson_dslash (same arguments, kernels and results), with every
 * buffer beyond `in` and `out` -- descriptor tables, the links packed from the
 * handle's canonical copy, the packed input and output fields -- kept in one
 * library-owned device array of WL_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds from its first call on that GPU until the process ends.  The
 * call issues no hipMalloc, hipFree or memset.  A lattice and nrhs whose packed
 * fields and links do not fit that array return WL_ERR_ARG before any device
 * work (about: links 8 V/2 x (link bytes) + 2 or 4 fields of nrhs V/2 x (site
 * bytes); 16^4 in FP64 recon-18 with one RHS fits, 24^4 in FP16 fits).  The
 * current device must be the handle's.  Every call on one GPU shares the
 * array: calls that overlap on one GPU (several streams or host threads) race,
 * so the caller orders them.  Asynchronous on `stream`. */
#define WL_NOALLOC_SCRATCH_BYTES (128u << 20)
wl_status wilson_dslash_noalloc(wl_gauge U, const double *in, double *out, int32_t nrhs, double kappa,
                                int32_t parity, int32_t dagger, wl_prec prec, int32_t recon, void *stream);

/* ---------------------------------------------------------------- solvers */

/* Solve D psi = eta (kappa normalisation) for nrhs right-hand sides by
 * even-odd preconditioned CG on the normal equations:
 *   b' = eta_e + kappa D_eo eta_o,  M = 1 - kappa^2 D_eo D_oe,
 *   CGNR on M^+ M x = M^+ b', psi_e = x, psi_o = eta_o + kappa D_oe psi_e.
 * Iterations run in the `sloppy` storage precision (FP32 arithmetic unless
 * WL_F64) with FP64 reliable updates: the solution accumulates in FP64 and the
 * residual b' - M x is recomputed in FP64 whenever the sloppy residual has
 * fallen by `delta` (0 < delta < 1; typical 0.1) since the last update.  The
 * solve stops when the FP64 residual is <= tol * |eta|.
 * eta, x: device, nrhs canonical fields; x holds the initial guess on entry
 * (zero it for none) and the solution on exit.  info: host array of nrhs.
 * A zero source gives x = 0, converged = 1.  On WL_ERR_NOCONV x holds the last
 * iterate and info is filled.  Synchronises `stream`. */
wl_status wilson_cg(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double tol,
                    int32_t maxiter, wl_prec sloppy, int32_t recon, double delta, wl_solve_info *info,
                    void *stream);

/* Solve D psi = eta as wilson_cg does, but with BiCGStab on the even-odd
 * Schur system M x = b' itself instead of CG on its normal equations: two
 * applications of M per iteration, complex BiCGStab scalars and dot products
 * in FP64, the same mixed-precision reliable updates (r replaced by the FP64
 * residual, rho recomputed) and the same stopping rule on the FP64 residual.
 * A breakdown (<rhat, M p> = 0 or |M s| = 0) or a non-finite sloppy value
 * restarts from the FP64 solution with a new shadow residual.  Arguments,
 * ownership and errors as in wilson_cg.  Synchronises `stream`. */
wl_status wilson_bicgstab(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double tol,
                          int32_t maxiter, wl_prec sloppy, int32_t recon, double delta, wl_solve_info *info,
                          void *stream);

/* Solve nsys independent systems (each its own gauge handle and geometry,
 * nrhs[i] right-hand sides, kappa[i]) together: every kernel launch of an
 * iteration covers all still-unconverged right-hand sides of all systems,
 * using device-resident per-system descriptors, and the iteration chunks are
 * replayed from a captured HIP graph.  eta[i], x[i]: device pointers as in
 * wilson_cg.  info: host array of sum(nrhs) entries, system-major.
 * Synchronises `stream`. */
wl_status wilson_cg_multi(int32_t nsys, const wl_gauge *U, const double *const *eta, double *const *x,
                          const int32_t *nrhs, const double *kappa, double tol, int32_t maxiter,
                          wl_prec sloppy, int32_t recon, double delta, wl_solve_info *info, void *stream);

/* ---------------------------------------------------------------- Wilson-clover */

/* The Wilson-clover operator (QUDA_DIRAC_CLOVER of Table 1) in the kappa
 * normalisation of the hop:  D = A - kappa H,  A(x) = 1 + i kappa c_sw
 * sum_{m<n} s_mn F_mn(x), s_mn = (i/2)[g_m, g_n], F_mn = (Q_mn - Q_mn^dagger)/8
 * with Q_mn(x) the four plaquettes of the m-n plane with a corner at x (each a
 * loop from x, m-direction first).  A is built on the GPU from the handle's
 * links on first use for each value of kappa c_sw and kept with the handle
 * (FP64, FP32 and FP16 copies of A and A^{-1}: 2 x 1008 bytes per site; FP16
 * and BF16 launches read the FP16 copy).  c_sw = 0
 * gives the Wilson operator.  Layouts, streams and errors as for the Wilson
 * entry points. */

/* out = D in (dagger: A in - kappa H^dagger in) on the whole lattice, nrhs
 * canonical fields; in and out must not overlap.  Asynchronous on `stream`. */
wl_status wilson_clover_dslash(wl_gauge U, const double *in, double *out, int32_t nrhs, double kappa, double csw,
                               int32_t dagger, wl_prec prec, int32_t recon, void *stream);

/* Solve D psi = eta as wilson_cg / wilson_bicgstab do, on the asymmetric Schur
 * complement M = A_ee - kappa^2 D_eo A_oo^{-1} D_oe with b' = eta_e +
 * kappa D_eo A_oo^{-1} eta_o and psi_o = A_oo^{-1} (eta_o + kappa D_oe psi_e);
 * the stop test and info are those of wilson_cg, with the clover operator.
 * Synchronises `stream`. */
wl_status wilson_clover_cg(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double csw,
                           double tol, int32_t maxiter, wl_prec sloppy, int32_t recon, double delta,
                           wl_solve_info *info, void *stream);
wl_status wilson_clover_bicgstab(wl_gauge U, const double *eta, double *x, int32_t nrhs, double kappa, double csw,
                                 double tol, int32_t maxiter, wl_prec sloppy, int32_t recon, double delta,
                                 wl_solve_info *info, void *stream);

/* ---------------------------------------------------------------- overlap sign */

/* out = eps(H_W) in ~= scale^{-1/2} H_W p(H_W^2 / scale) in on the whole
 * lattice, for nrhs canonical fields (device).  p is the Chebyshev interpolant
 * of degree `degree` of x^{-1/2} on [lo, hi] at the degree+1 first-kind
 * Chebyshev nodes, applied by the Clenshaw recurrence.  H_W = g5 D_m(-rho)
 * (mass normalisation, kappa = 1/(8 - 2 rho)).  scale > 0 is the number the
 * spectrum of H_W^2 is divided by; scale <= 0 asks the library to estimate
 * 1.02 x lambda_max(H_W^2) by power iteration first.  prec is the storage
 * precision of the iteration (WL_F64 or WL_F32).  Synchronises `stream`. */
wl_status overlap_sign_cheb(wl_gauge U, const double *in, double *out, int32_t nrhs, double rho,
                            int32_t degree, double lo, double hi, double scale, wl_prec prec,
                            int32_t recon, int32_t nev, const double *evecs, const double *evals,
                            void *stream);

/* Low-mode deflation (the last three arguments of overlap_sign_cheb,
 * overlap_dslash and overlap_cg): nev in [0, 64] orthonormal eigenvectors of
 * H_W (evecs: device, nev canonical whole-lattice fields) with their
 * eigenvalues (evals: host, nev doubles).  The sign function then acts exactly
 * on their span and by the polynomial on its orthogonal complement:
 *   eps(H_W) v = sum_i sign(lambda_i) xi_i <xi_i, v> + eps_poly(H_W) (v - sum_i xi_i <xi_i, v>),
 * so the window [lo, hi] only has to cover the rest of the spectrum.  nev = 0
 * (evecs, evals may be NULL) is the plain polynomial.  wl_hw_eigs computes
 * such eigenpairs. */

/* The nev eigenpairs of H_W (m0 = -rho) of smallest |lambda|, by
 * Chebyshev-filtered subspace iteration on H_W^2 in FP64 with a block of
 * nblock vectors (nev <= nblock <= 64): each pass applies T_degree of H_W^2
 * mapped so that the window [a, 1] of H_W^2 / scale is damped (a = the
 * block's largest Ritz value, 0.05 at first), orthonormalises the block and
 * takes Ritz pairs of H_W.  scale <= 0: 1.02 x a power-iteration estimate of
 * lambda_max(H_W^2).  Stops when every wanted residual |H_W xi - lambda xi|
 * <= tol or after maxiter passes (WL_ERR_NOCONV, results filled).  evecs:
 * device, nev canonical fields (orthonormal, ordered by |lambda|); evals,
 * resid: host, nev doubles; iters: host (may be NULL).  Synchronises. */
wl_status wl_hw_eigs(wl_gauge U, double rho, int32_t nev, int32_t nblock, int32_t degree, double tol,
                     int32_t maxiter, double scale, double *evecs, double *evals, double *resid, int32_t *iters,
                     void *stream);

/* ---------------------------------------------------------------- overlap operator */

/* out = D_ov(m) in, the overlap operator of the GWU-code inverter (Sections 1
 * and 3), with the sign function of overlap_sign_cheb:
 *   D_ov(m)        = (rho + m/2) + (rho - m/2) g5 eps(H_W)
 *   D_ov(m)^dagger = (rho + m/2) + (rho - m/2) eps(H_W) g5      (dagger != 0)
 * Whole lattice, nrhs canonical fields (device), in and out must not overlap.
 * mass in [0, 2 rho); degree, lo, hi, scale as for overlap_sign_cheb (scale <= 0:
 * estimated from in's first field).  prec WL_F64 or WL_F32.  One call costs one
 * sign-function evaluation: 2 (degree + 1) + 1 applications of H_W.
 * Synchronises `stream`. */
wl_status overlap_dslash(wl_gauge U, const double *in, double *out, int32_t nrhs, double rho, double mass,
                         int32_t degree, double lo, double hi, double scale, int32_t dagger, wl_prec prec,
                         int32_t recon, int32_t nev, const double *evecs, const double *evals, void *stream);

/* Solve D_ov(m) x = eta for nrhs canonical fields (device; x holds the initial
 * guess on entry and the solution on exit; eta and x must not overlap).  CG on
 * the normal equations with the residual of the original system tracked, in a
 * defect-correction loop: the FP64 residual eta - D_ov x is recomputed with the
 * FP64 operator, an inner CG in the working precision `sloppy` (WL_F64 or
 * WL_F32) reduces it by the factor `delta` in (0, 1) (straight to the
 * tolerance when sloppy is WL_F64), and the correction is added to the FP64 x.
 * Stops when |eta - D_ov x| <= tol |eta| with the FP64 operator.  mass must be
 * > 0 (D_ov(0) has exact zero modes).  maxiter bounds the inner iterations in
 * total.  info: host array of nrhs entries; iters = inner iterations,
 * reliable_updates = recomputed residuals after the first, true_resid = the
 * final FP64 relative residual.  A zero source gives x = 0.  Returns
 * WL_ERR_NOCONV with x = the best iterate when tol is not reached.
 * Synchronises `stream`. */
wl_status overlap_cg(wl_gauge U, const double *eta, double *x, int32_t nrhs, double rho, double mass,
                     int32_t degree, double lo, double hi, double scale, double tol, int32_t maxiter,
                     wl_prec sloppy, int32_t recon, double delta, int32_t nev, const double *evecs,
                     const double *evals, wl_solve_info *info, void *stream);

/* Largest eigenvalue of H_W^2 (m0 = -rho) estimated by `iters` steps of power
 * iteration from the canonical field v0 (device); FP64.  Synchronises. */
wl_status wl_hw2_lmax(wl_gauge U, double rho, const double *v0, int32_t iters, double *lmax, void *stream);

/* ---------------------------------------------------------------- errors */

const char *wl_status_string(wl_status s);
const char *wl_last_error(void);

/* ---------------------------------------------------------------- measurement */

/* Time the single-parity hop kernel on library-owned packed fields (no
 * conversion inside the timed region): `reps` back-to-back launches on
 * `stream`, measured with HIP events on that stream.  nsets >= 1 independent
 * (links, in, out) sets are rotated so that consecutive launches do not find
 * their operands in the caches (cold protocol; its launch configuration is
 * tuned on rotated launches too) -- nsets = 1 is the warm protocol of a
 * solver, with the solver's tuned configuration.  Returns the mean seconds
 * per launch. */
wl_status wl_bench_dslash(wl_gauge U, wl_prec prec, int32_t recon, int32_t nrhs, int32_t parity,
                          int32_t nsets, int32_t reps, double *seconds_per_call, void *stream);

/* Time a plain device copy of `bytes` bytes (read + write), the measured
 * bandwidth reference for the roofline; mean seconds per launch of `reps`
 * back-to-back launches (after one untimed launch) on library-owned buffers.
 * mode 0: non-temporal loads and stores (the roofline reference and the
 * traffic-counter calibration); 1: ordinary loads and stores, so that
 * operands that fit the last-level cache are served from it; 2: ordinary
 * loads only (`bytes` read per launch, nothing written).  WL_ERR_ARG for
 * bytes < 1024, reps < 1 or another mode. */
wl_status wl_bench_copy(int64_t bytes, int32_t reps, int32_t mode, double *seconds_per_call, void *stream);

/* Per-kernel timing of the library's own hop launches: when enabled, every
 * hop launch outside graph capture drains its stream and is dispatched with
 * start/end HIP events that the dispatch itself records (dispatch to
 * completion), and its blocks store readings of the device's constant-rate
 * steady clock at their start and end, whose span (first block start to last
 * block end) is the kernel's own duration.  Solvers run without graphs while
 * timing is on.  wl_prof_read returns launches, total event milliseconds,
 * algorithmic GB and total kernel milliseconds of the timed launches since
 * the last read and resets the counters. */
wl_status wl_prof_enable(int32_t on);
wl_status wl_prof_read(int64_t *hop_launches, double *hop_ms, double *hop_gbytes, double *hop_kernel_ms);

/* Restrict that timing to hop launches of one storage precision (a wl_prec),
 * or -1 for all (the default). */
wl_status wl_prof_select(int32_t prec);

/* Algorithmic bytes per output site of one single-parity hop launch for a
 * storage precision, compression and RHS count: 8 links shared by the nrhs
 * right-hand sides, plus one input and one output spinor per RHS. */
double wl_hop_bytes_per_site(wl_prec prec, int32_t recon, int32_t nrhs);

#ifdef __cplusplus
}
#endif

#endif /* WILSON_MI355X_H */
