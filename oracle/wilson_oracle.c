/*
 * wilson_oracle.c -- plain, slow FP64 CPU reference for the Wilson-Dirac
 * inverter path (dslash, even-odd CG on the normal equations, Chebyshev
 * sign function, overlap operator and its CG solve, clover term).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * The paper (Lattice QCD package GWU-code and QUDA with HIP, LATTICE2019)
 * names the Wilson-Dirac operator (Table 1, QUDA_DIRAC_WILSON), its D-slash
 * kernel with SU(3) links (Table 2 and its caption), and the overlap fermion
 * inverter of GWU-code (Sections 1 and 3), but writes down no formula.  The
 * definitions below are the standard lattice-QCD ones; each convention choice
 * is one of the readings listed in the design notes.
 *
 * Conventions (complex128, AoS, the canonical layout of the library ABI):
 *   site s = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2, even = 0.
 *   U[s][mu][a][b]: U_mu(x), 3x3 row-major.  psi[s][spin][colour].
 *   Gamma matrices in the DeGrand-Rossi basis (g5 = gx gy gz gt = diag(1,1,-1,-1)).
 *   Hopping term (one output site x):
 *     (H psi)(x) = sum_mu  b (1 - g_mu) U_mu(x) psi(x+mu)
 *                        + b (1 + g_mu) U_mu(x-mu)^dagger psi(x-mu)
 *   with b = -1 on a hop that crosses the time boundary when the time
 *   direction is antiperiodic, else +1.  The adjoint H^dagger is the same sum
 *   with (1 - g_mu) and (1 + g_mu) swapped.
 *   Wilson operator, kappa normalisation:   D_k = 1 - kappa H
 *   mass normalisation:  D_m(m0) = (4 + m0) - H/2 = D_k / (2 kappa), kappa = 1/(8 + 2 m0)
 *   overlap kernel:      H_W = g5 D_m(-rho)
 *
 * Spin is applied with full 4x4 matrix products (no half-spinor projection);
 * colour with full 3x3 products.  OpenMP only splits independent sites.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---- lattice geometry -------------------------------------------------- */

typedef struct {
    int L[4];
    int antiperiodic_t;
    long V;
} lattice;

static lattice make_lattice(const int32_t *L, int32_t antiperiodic_t)
{
    lattice g;
    g.V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = L[mu];
        g.V *= L[mu];
    }
    g.antiperiodic_t = antiperiodic_t;
    return g;
}

static void site_coords(const lattice *g, long s, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % g->L[mu]);
        s /= g->L[mu];
    }
}

static long site_index(const lattice *g, const int c[4])
{
    return c[0] + (long)g->L[0] * (c[1] + (long)g->L[1] * (c[2] + (long)g->L[2] * c[3]));
}

static int site_parity(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* neighbour of c one step along +mu (dir = +1) or -mu (dir = -1); *bc is the
 * boundary factor of that hop */
static long neighbour(const lattice *g, const int c[4], int mu, int dir, double *bc)
{
    int n[4] = {c[0], c[1], c[2], c[3]};
    n[mu] += dir;
    *bc = 1.0;
    if (n[mu] == g->L[mu]) {
        n[mu] = 0;
        if (mu == 3 && g->antiperiodic_t) *bc = -1.0;
    } else if (n[mu] < 0) {
        n[mu] = g->L[mu] - 1;
        if (mu == 3 && g->antiperiodic_t) *bc = -1.0;
    }
    return site_index(g, n);
}

/* ---- gamma matrices (DeGrand-Rossi) ------------------------------------ */

static void gamma_matrix(int mu, cplx gm[4][4])
{
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) gm[i][j] = 0;
    switch (mu) {
    case 0: /* gamma_x */
        gm[0][3] = I; gm[1][2] = I; gm[2][1] = -I; gm[3][0] = -I;
        break;
    case 1: /* gamma_y */
        gm[0][3] = -1; gm[1][2] = 1; gm[2][1] = 1; gm[3][0] = -1;
        break;
    case 2: /* gamma_z */
        gm[0][2] = I; gm[1][3] = -I; gm[2][0] = -I; gm[3][1] = I;
        break;
    case 3: /* gamma_t */
        gm[0][2] = 1; gm[1][3] = 1; gm[2][0] = 1; gm[3][1] = 1;
        break;
    case 4: /* gamma_5 = gx gy gz gt */
        gm[0][0] = 1; gm[1][1] = 1; gm[2][2] = -1; gm[3][3] = -1;
        break;
    }
}

void or_gamma(int32_t mu, double *out /* 4x4 complex, row-major */)
{
    cplx gm[4][4];
    gamma_matrix(mu, gm);
    memcpy(out, gm, sizeof(gm));
}

/* ---- the hopping term --------------------------------------------------- */

/* acc += b * P * (W psi_y), where W is U (adj = 0) or U^dagger (adj = 1) and
 * P is the 4x4 spin matrix 1 + sgn*gamma_mu */
static void accumulate_hop(cplx acc[4][3], const cplx *Umat, int adj, const cplx *psi_y,
                           cplx gm[4][4], double sgn, double b)
{
    cplx chi[4][3];
    for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
            cplx v = 0;
            for (int bb = 0; bb < 3; ++bb) {
                cplx u = adj ? conj(Umat[bb * 3 + a]) : Umat[a * 3 + bb];
                v += u * psi_y[sp * 3 + bb];
            }
            chi[sp][a] = v;
        }
    for (int i = 0; i < 4; ++i)
        for (int a = 0; a < 3; ++a) {
            cplx v = 0;
            for (int j = 0; j < 4; ++j) {
                cplx pij = (i == j ? 1.0 : 0.0) + sgn * gm[i][j];
                v += pij * chi[j][a];
            }
            acc[i][a] += b * v;
        }
}

/* out = H in (dagger = 0) or H^dagger in (dagger = 1) at the output sites of
 * the given parity (0 even, 1 odd, -1 all); other output sites are set to 0.
 * With out_parity = p the result reads only the opposite-parity sites of in,
 * which is the single-parity hop D_{p,1-p}.  in and out hold nrhs fields. */
void or_hop(const int32_t *L, int32_t antiperiodic_t, const double *U_, const double *in_,
            double *out_, int32_t nrhs, int32_t out_parity, int32_t dagger)
{
    lattice g = make_lattice(L, antiperiodic_t);
    const cplx *U = (const cplx *)U_;
    cplx gms[4][4][4];
    for (int mu = 0; mu < 4; ++mu) gamma_matrix(mu, gms[mu]);
    /* forward hop carries 1 - g_mu, backward 1 + g_mu; the adjoint swaps them */
    const double sfwd = dagger ? +1.0 : -1.0;
    const double sbwd = -sfwd;
    for (int r = 0; r < nrhs; ++r) {
        const cplx *in = (const cplx *)in_ + (size_t)r * g.V * 12;
        cplx *out = (cplx *)out_ + (size_t)r * g.V * 12;
#pragma omp parallel for schedule(static)
        for (long s = 0; s < g.V; ++s) {
            int c[4];
            site_coords(&g, s, c);
            cplx acc[4][3] = {{0}};
            if (out_parity < 0 || site_parity(c) == out_parity) {
                for (int mu = 0; mu < 4; ++mu) {
                    double b;
                    long yf = neighbour(&g, c, mu, +1, &b);
                    accumulate_hop(acc, U + (s * 4 + mu) * 9, 0, in + yf * 12, gms[mu], sfwd, b);
                    long yb = neighbour(&g, c, mu, -1, &b);
                    accumulate_hop(acc, U + (yb * 4 + mu) * 9, 1, in + yb * 12, gms[mu], sbwd, b);
                }
            }
            for (int i = 0; i < 4; ++i)
                for (int a = 0; a < 3; ++a) out[s * 12 + i * 3 + a] = acc[i][a];
        }
    }
}

/* ---- small vector helpers (n complex numbers) -------------------------- */

/* reductions run serially, in index order, so that results do not depend on
 * the thread count */
static double vnorm2(const cplx *a, long n)
{
    double s = 0;
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

static cplx vdot(const cplx *a, const cplx *b, long n) /* sum conj(a) b */
{
    double re = 0, im = 0;
    for (long i = 0; i < n; ++i) {
        cplx p = conj(a[i]) * b[i];
        re += creal(p);
        im += cimag(p);
    }
    return re + I * im;
}

/* y = a*x + b*y */
static void vaxpby(cplx a, const cplx *x, cplx b, cplx *y, long n)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) y[i] = a * x[i] + b * y[i];
}

static void vgamma5(const cplx *in, cplx *out, long V) /* may alias */
{
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s)
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                double g5 = sp < 2 ? 1.0 : -1.0;
                out[s * 12 + sp * 3 + a] = g5 * in[s * 12 + sp * 3 + a];
            }
}

/* zero the sites of the given parity */
static void vzero_parity(const lattice *g, cplx *v, int parity)
{
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g->V; ++s) {
        int c[4];
        site_coords(g, s, c);
        if (site_parity(c) == parity)
            for (int k = 0; k < 12; ++k) v[s * 12 + k] = 0;
    }
}

/* ---- full operators ----------------------------------------------------- */

/* out = D_k in = in - kappa H in (dagger: in - kappa H^dagger in), whole lattice */
void or_wilson(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *in_,
               double *out_, int32_t nrhs, double kappa, int32_t dagger)
{
    lattice g = make_lattice(L, antiperiodic_t);
    or_hop(L, antiperiodic_t, U, in_, out_, nrhs, -1, dagger);
    long n = g.V * 12 * (long)nrhs;
    vaxpby(1.0, (const cplx *)in_, -kappa, (cplx *)out_, n);
}

/* out = H_W in = g5 ((4 + m0) in - H in / 2), m0 = -rho, whole lattice */
void or_overlap_kernel(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *in_,
                       double *out_, int32_t nrhs, double rho)
{
    lattice g = make_lattice(L, antiperiodic_t);
    or_hop(L, antiperiodic_t, U, in_, out_, nrhs, -1, 0);
    long n = g.V * 12 * (long)nrhs;
    vaxpby(4.0 - rho, (const cplx *)in_, -0.5, (cplx *)out_, n);
    vgamma5((const cplx *)out_, (cplx *)out_, g.V * nrhs);
}

/* ---- even-odd Schur operator ------------------------------------------- */
/* Vectors live on the whole lattice with zeros on the odd sites.
 *   D_eo = P_e H P_o,  D_oe = P_o H P_e,  M = 1 - kappa^2 D_eo D_oe   (even sites)
 *   M^dagger = 1 - kappa^2 D_oe^dagger D_eo^dagger, where D_oe^dagger = P_e H^dagger P_o */

typedef struct {
    const int32_t *L;
    int32_t tap;
    const double *U;
    double kappa;
    cplx *tmp; /* one whole-lattice field */
} schur_op;

static void schur_apply(const schur_op *op, const cplx *in, cplx *out, int dagger, long V)
{
    or_hop(op->L, op->tap, op->U, (const double *)in, (double *)op->tmp, 1, 1, dagger);
    or_hop(op->L, op->tap, op->U, (const double *)op->tmp, (double *)out, 1, 0, dagger);
    vaxpby(1.0, in, -op->kappa * op->kappa, out, V * 12);
}

/* Even-odd CG on the normal equations (CGNR) for D_k psi = eta.
 *   b' = eta_e + kappa D_eo eta_o;  solve M x = b' through M^dagger M x = M^dagger b',
 *   tracking the residual rt = b' - M x of the original system, which CGNR
 *   updates for free from q = M p.  Stop when |rt| <= tol |eta| holds for the
 *   recomputed rt = b' - M x.  Then psi_e = x, psi_o = eta_o + kappa D_oe psi_e.
 * x holds the initial guess on entry (its odd sites are ignored) and the whole-
 * lattice solution on exit.  Returns 0 when converged, 1 otherwise.
 * iters_out: iterations taken; resid_out: |eta - D_k psi| / |eta| with the
 * whole-lattice operator.  nrhs systems are solved one after the other;
 * iters_out and resid_out have nrhs entries. */
int32_t or_cg_eo(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *eta_,
                 double *x_, int32_t nrhs, double kappa, double tol, int32_t maxiter,
                 int32_t *iters_out, double *resid_out)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long V = g.V, n = V * 12;
    cplx *bp = malloc(sizeof(cplx) * n), *rt = malloc(sizeof(cplx) * n);
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    int32_t status = 0;
    schur_op op = {L, antiperiodic_t, U, kappa, tmp};

    for (int rh = 0; rh < nrhs; ++rh) {
        const cplx *eta = (const cplx *)eta_ + (size_t)rh * n;
        cplx *x = (cplx *)x_ + (size_t)rh * n;
        double eta_norm = sqrt(vnorm2(eta, n));
        int it = 0, converged = 0;

        /* b' = eta_e + kappa D_eo eta_o */
        or_hop(L, antiperiodic_t, U, (const double *)eta, (double *)bp, 1, 0, 0);
        vaxpby(1.0, eta, kappa, bp, n);
        vzero_parity(&g, bp, 1);
        vzero_parity(&g, x, 1);

        if (eta_norm == 0.0) {
            memset(x, 0, sizeof(cplx) * n);
            iters_out[rh] = 0;
            resid_out[rh] = 0.0;
            continue;
        }
        /* rt = b' - M x;  r = M^dagger rt;  p = r;  gamma = |r|^2 */
        schur_apply(&op, x, q, 0, V);
        memcpy(rt, bp, sizeof(cplx) * n);
        vaxpby(-1.0, q, 1.0, rt, n);
        schur_apply(&op, rt, r, 1, V);
        memcpy(p, r, sizeof(cplx) * n);
        double gam = vnorm2(r, n);

        while (it < maxiter) {
            if (sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
                /* confirm on the recomputed residual */
                schur_apply(&op, x, q, 0, V);
                memcpy(rt, bp, sizeof(cplx) * n);
                vaxpby(-1.0, q, 1.0, rt, n);
                if (sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
                    converged = 1;
                    break;
                }
                schur_apply(&op, rt, r, 1, V);
                gam = vnorm2(r, n);
                memcpy(p, r, sizeof(cplx) * n);
            }
            schur_apply(&op, p, q, 0, V); /* q = M p */
            double alpha = gam / vnorm2(q, n);
            vaxpby(alpha, p, 1.0, x, n);   /* x += alpha p */
            vaxpby(-alpha, q, 1.0, rt, n); /* rt -= alpha q */
            schur_apply(&op, rt, r, 1, V); /* s = M^dagger rt */
            double gam_new = vnorm2(r, n);
            vaxpby(1.0, r, gam_new / gam, p, n); /* p = s + beta p */
            gam = gam_new;
            ++it;
        }
        if (!converged && sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
            schur_apply(&op, x, q, 0, V);
            memcpy(rt, bp, sizeof(cplx) * n);
            vaxpby(-1.0, q, 1.0, rt, n);
            converged = sqrt(vnorm2(rt, n)) <= tol * eta_norm;
        }

        /* psi_o = eta_o + kappa D_oe psi_e */
        or_hop(L, antiperiodic_t, U, (const double *)x, (double *)tmp, 1, 1, 0);
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; ++s) {
            int c[4];
            site_coords(&g, s, c);
            if (site_parity(c) == 1)
                for (int k = 0; k < 12; ++k) x[s * 12 + k] = eta[s * 12 + k] + kappa * tmp[s * 12 + k];
        }

        /* independent true residual with the whole-lattice operator */
        or_wilson(L, antiperiodic_t, U, (const double *)x, (double *)tmp, 1, kappa, 0);
        vaxpby(1.0, eta, -1.0, tmp, n);
        iters_out[rh] = it;
        resid_out[rh] = sqrt(vnorm2(tmp, n)) / eta_norm;
        if (!converged) status = 1;
    }
    free(bp); free(rt); free(r); free(p); free(q); free(tmp);
    return status;
}

/* ---- Chebyshev approximation of the sign function ----------------------- */

/* Coefficients of the Chebyshev interpolant of f(x) = x^{-1/2} on [lo, hi],
 * degree d (N = d + 1 terms), at the N first-kind Chebyshev nodes:
 *   theta_k = pi (k + 1/2) / N,  x_k = (hi - lo)/2 cos theta_k + (hi + lo)/2
 *   c_j = (2/N) sum_k f(x_k) cos(j theta_k),  p(x) = c_0/2 + sum_{j>=1} c_j T_j(y(x))
 * with y(x) = (2x - hi - lo) / (hi - lo). */
void or_cheb_coeffs(int32_t degree, double lo, double hi, double *c)
{
    int N = degree + 1;
    for (int j = 0; j < N; ++j) {
        double s = 0;
        for (int k = 0; k < N; ++k) {
            double th = M_PI * (k + 0.5) / N;
            double xk = 0.5 * (hi - lo) * cos(th) + 0.5 * (hi + lo);
            s += cos(j * th) / sqrt(xk);
        }
        c[j] = 2.0 * s / N;
    }
}

/* Scalar evaluation of that polynomial at x, by the same Clenshaw recurrence. */
double or_cheb_eval(int32_t degree, const double *c, double lo, double hi, double x)
{
    double y = (2.0 * x - hi - lo) / (hi - lo);
    double b1 = 0, b2 = 0;
    for (int j = degree; j >= 1; --j) {
        double b0 = 2.0 * y * b1 - b2 + c[j];
        b2 = b1;
        b1 = b0;
    }
    return y * b1 - b2 + 0.5 * c[0];
}

/* out = eps(H_W) in ~= s^{-1/2} H_W p(H_W^2 / s) in, whole lattice, nrhs fields.
 * p is the degree-d Chebyshev interpolant of x^{-1/2} on [lo, hi]; it is
 * applied by the Clenshaw recurrence with Y = (2 H_W^2 / s - hi - lo)/(hi - lo):
 *   b_{N} = b_{N+1} = 0,  b_j = 2 Y b_{j+1} - b_{j+2} + c_j v  (j = N-1 .. 1),
 *   p v = Y b_1 - b_2 + c_0 v / 2. */
void or_sign_cheb(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *in_,
                  double *out_, int32_t nrhs, double rho, int32_t degree, double lo, double hi,
                  double scale)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long n = g.V * 12;
    int N = degree + 1;
    double *c = malloc(sizeof(double) * N);
    or_cheb_coeffs(degree, lo, hi, c);
    cplx *b0 = malloc(sizeof(cplx) * n), *b1 = malloc(sizeof(cplx) * n);
    cplx *b2 = malloc(sizeof(cplx) * n), *w = malloc(sizeof(cplx) * n);
    cplx *yb = malloc(sizeof(cplx) * n);
    const double ay = 2.0 / ((hi - lo) * scale), by = -(hi + lo) / (hi - lo);

    for (int r = 0; r < nrhs; ++r) {
        const cplx *v = (const cplx *)in_ + (size_t)r * n;
        cplx *out = (cplx *)out_ + (size_t)r * n;
        memset(b1, 0, sizeof(cplx) * n); /* b_{j+1} */
        memset(b2, 0, sizeof(cplx) * n); /* b_{j+2} */
        for (int j = N - 1; j >= 1; --j) {
            /* yb = Y b1 = ay H_W (H_W b1) + by b1 */
            or_overlap_kernel(L, antiperiodic_t, U, (const double *)b1, (double *)w, 1, rho);
            or_overlap_kernel(L, antiperiodic_t, U, (const double *)w, (double *)yb, 1, rho);
            vaxpby(by, b1, ay, yb, n);
            /* b0 = 2 yb - b2 + c_j v */
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) b0[i] = 2.0 * yb[i] - b2[i] + c[j] * v[i];
            cplx *t = b2;
            b2 = b1;
            b1 = b0;
            b0 = t;
        }
        /* p v = Y b1 - b2 + c_0 v / 2 */
        or_overlap_kernel(L, antiperiodic_t, U, (const double *)b1, (double *)w, 1, rho);
        or_overlap_kernel(L, antiperiodic_t, U, (const double *)w, (double *)yb, 1, rho);
        vaxpby(by, b1, ay, yb, n);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) w[i] = yb[i] - b2[i] + 0.5 * c[0] * v[i];
        /* out = s^{-1/2} H_W (p v) */
        or_overlap_kernel(L, antiperiodic_t, U, (const double *)w, (double *)out, 1, rho);
        vaxpby(0.0, out, 1.0 / sqrt(scale), out, n);
    }
    free(c); free(b0); free(b1); free(b2); free(w); free(yb);
}

/* ---- low-mode deflation of the sign function ----------------------------- */
/* With nev orthonormal eigenvectors xi_i of H_W (eigenvalues lambda_i) the
 * sign function acts exactly on their span and by the polynomial on the rest:
 *   eps(H_W) v = sum_i sign(lambda_i) xi_i <xi_i, v> + eps_poly(H_W) (v - sum_i xi_i <xi_i, v>)
 * evecs: nev whole-lattice fields; nev = 0 is the plain polynomial. */
static void sign_deflated(const int32_t *L, int32_t antiperiodic_t, const double *U, const cplx *v, cplx *out,
                          double rho, int32_t degree, double lo, double hi, double scale, int32_t nev,
                          const double *evecs_, const double *evals)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long n = g.V * 12;
    if (nev <= 0) {
        or_sign_cheb(L, antiperiodic_t, U, (const double *)v, (double *)out, 1, rho, degree, lo, hi, scale);
        return;
    }
    const cplx *xi = (const cplx *)evecs_;
    cplx *w = malloc(sizeof(cplx) * n), *c = malloc(sizeof(cplx) * nev);
    memcpy(w, v, sizeof(cplx) * n);
    for (int i = 0; i < nev; ++i) {
        c[i] = vdot(xi + (size_t)i * n, v, n);
        vaxpby(-c[i], xi + (size_t)i * n, 1.0, w, n);
    }
    or_sign_cheb(L, antiperiodic_t, U, (const double *)w, (double *)out, 1, rho, degree, lo, hi, scale);
    for (int i = 0; i < nev; ++i) vaxpby((evals[i] > 0 ? 1.0 : -1.0) * c[i], xi + (size_t)i * n, 1.0, out, n);
    free(w); free(c);
}

/* the deflated sign function on nrhs fields */
void or_sign_cheb_defl(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *in_,
                       double *out_, int32_t nrhs, double rho, int32_t degree, double lo, double hi,
                       double scale, int32_t nev, const double *evecs, const double *evals)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long n = g.V * 12;
    for (int r = 0; r < nrhs; ++r)
        sign_deflated(L, antiperiodic_t, U, (const cplx *)in_ + (size_t)r * n, (cplx *)out_ + (size_t)r * n, rho,
                      degree, lo, hi, scale, nev, evecs, evals);
}

/* ---- overlap operator (GWU-code's inverter, Sections 1 and 3) ----------- */
/* Neuberger's overlap operator with bare mass m, built on the approximate
 * sign function above:
 *   D_ov(m) = (rho + m/2) + (rho - m/2) g5 eps(H_W)
 *   D_ov(m)^dagger = (rho + m/2) + (rho - m/2) eps(H_W) g5      (eps is Hermitian)
 * whole lattice, nrhs fields. */
void or_overlap(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *in_,
                double *out_, int32_t nrhs, double rho, double mass, int32_t degree, double lo,
                double hi, double scale, int32_t dagger, int32_t nev, const double *evecs,
                const double *evals)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long n = g.V * 12;
    const double a = rho + 0.5 * mass, b = rho - 0.5 * mass;
    cplx *t = malloc(sizeof(cplx) * n), *w = malloc(sizeof(cplx) * n);
    for (int r = 0; r < nrhs; ++r) {
        const cplx *v = (const cplx *)in_ + (size_t)r * n;
        cplx *out = (cplx *)out_ + (size_t)r * n;
        if (dagger) {
            vgamma5(v, t, g.V);
            sign_deflated(L, antiperiodic_t, U, t, w, rho, degree, lo, hi, scale, nev, evecs, evals);
        } else {
            sign_deflated(L, antiperiodic_t, U, v, t, rho, degree, lo, hi, scale, nev, evecs, evals);
            vgamma5(t, w, g.V);
        }
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) out[i] = a * v[i] + b * w[i];
    }
    free(t); free(w);
}

/* Overlap solve D_ov(m) x = eta by CG on the normal equations (CGNR), tracking
 * the residual rt = eta - D x of the original system:
 *   rt = eta - D x;  s = D^dagger rt;  p = s;  gamma = |s|^2
 *   repeat:  q = D p;  alpha = gamma / |q|^2;  x += alpha p;  rt -= alpha q;
 *            stop when |rt| <= tol |eta| holds for the recomputed rt;
 *            s = D^dagger rt;  p = s + (|s|^2 / gamma) p
 * x holds the initial guess on entry.  Returns 0 when every system converged.
 * resid_out: |eta - D x| / |eta| with the same operator, recomputed. */
int32_t or_overlap_cg(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *eta_,
                      double *x_, int32_t nrhs, double rho, double mass, int32_t degree, double lo,
                      double hi, double scale, double tol, int32_t maxiter, int32_t nev,
                      const double *evecs, const double *evals, int32_t *iters_out, double *resid_out)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long n = g.V * 12;
    cplx *rt = malloc(sizeof(cplx) * n), *sv = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    int32_t status = 0;
#define OV_APPLY(in, out, dag) \
    or_overlap(L, antiperiodic_t, U, (const double *)(in), (double *)(out), 1, rho, mass, degree, lo, hi, scale, dag, \
               nev, evecs, evals)
    for (int rh = 0; rh < nrhs; ++rh) {
        const cplx *eta = (const cplx *)eta_ + (size_t)rh * n;
        cplx *x = (cplx *)x_ + (size_t)rh * n;
        double eta_norm = sqrt(vnorm2(eta, n));
        int it = 0, converged = 0;
        if (eta_norm == 0.0) {
            memset(x, 0, sizeof(cplx) * n);
            iters_out[rh] = 0;
            resid_out[rh] = 0.0;
            continue;
        }
        OV_APPLY(x, q, 0);
        memcpy(rt, eta, sizeof(cplx) * n);
        vaxpby(-1.0, q, 1.0, rt, n);
        OV_APPLY(rt, sv, 1);
        memcpy(p, sv, sizeof(cplx) * n);
        double gam = vnorm2(sv, n);
        while (it < maxiter) {
            if (sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
                OV_APPLY(x, q, 0);
                memcpy(rt, eta, sizeof(cplx) * n);
                vaxpby(-1.0, q, 1.0, rt, n);
                if (sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
                    converged = 1;
                    break;
                }
                OV_APPLY(rt, sv, 1);
                gam = vnorm2(sv, n);
                memcpy(p, sv, sizeof(cplx) * n);
            }
            OV_APPLY(p, q, 0);
            double alpha = gam / vnorm2(q, n);
            vaxpby(alpha, p, 1.0, x, n);
            vaxpby(-alpha, q, 1.0, rt, n);
            OV_APPLY(rt, sv, 1);
            double gam_new = vnorm2(sv, n);
            vaxpby(1.0, sv, gam_new / gam, p, n);
            gam = gam_new;
            ++it;
        }
        OV_APPLY(x, q, 0);
        memcpy(rt, eta, sizeof(cplx) * n);
        vaxpby(-1.0, q, 1.0, rt, n);
        resid_out[rh] = sqrt(vnorm2(rt, n)) / eta_norm;
        iters_out[rh] = it;
        if (!(converged || resid_out[rh] <= tol)) status = 1;
    }
#undef OV_APPLY
    free(rt); free(sv); free(p); free(q);
    return status;
}

/* Largest eigenvalue of H_W^2 by power iteration from the start vector v0
 * (Rayleigh quotient after iters steps). */
double or_hw2_lmax(const int32_t *L, int32_t antiperiodic_t, const double *U, double rho,
                   const double *v0, int32_t iters)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long n = g.V * 12;
    cplx *v = malloc(sizeof(cplx) * n), *w = malloc(sizeof(cplx) * n), *u = malloc(sizeof(cplx) * n);
    memcpy(v, v0, sizeof(cplx) * n);
    double lam = 0;
    double nv = sqrt(vnorm2(v, n));
    vaxpby(0.0, v, 1.0 / nv, v, n);
    for (int it = 0; it < iters; ++it) {
        or_overlap_kernel(L, antiperiodic_t, U, (const double *)v, (double *)u, 1, rho);
        or_overlap_kernel(L, antiperiodic_t, U, (const double *)u, (double *)w, 1, rho);
        lam = creal(vdot(v, w, n));
        double nw = sqrt(vnorm2(w, n));
        for (long i = 0; i < n; ++i) v[i] = w[i] / nw;
    }
    free(v); free(w); free(u);
    return lam;
}

/* ---- clover term (QUDA_DIRAC_CLOVER of Table 1) ------------------------ */
/* Sheikholeslami-Wohlert term in the normalisation of the hopping term above
 * (forward hop 1 - g_mu), with the clover-leaf field strength:
 *   Q_mn(x) = sum of the four plaquettes of the m-n plane that start and end
 *             at x, each traversed m-direction first (counter-clockwise)
 *   F_mn(x) = (Q_mn(x) - Q_mn(x)^dagger) / 8            (anti-Hermitian)
 *   s_mn    = (i/2) [g_m, g_n]
 *   D_mass  = (4 + m0) - H/2 + (i c_sw / 2) sum_{m<n} s_mn F_mn
 *   D_k     = 2 kappa D_mass = A - kappa H,  A(x) = 1 + i kappa c_sw sum_{m<n} s_mn F_mn(x)
 * A(x) is a Hermitian 12 x 12 matrix at each site (spin-major, colour-minor),
 * stored as A[s][12][12] complex.  Gauge links are periodic in every
 * direction; the fermion boundary factor of the hop does not enter Q. */

/* c = op(a) op(b) for 3x3 complex matrices, op = dagger when the flag is set */
static void m3_mul(const cplx *a, int ad, const cplx *b, int bd, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx v = 0;
            for (int k = 0; k < 3; ++k) {
                cplx x = ad ? conj(a[k * 3 + i]) : a[i * 3 + k];
                cplx y = bd ? conj(b[j * 3 + k]) : b[k * 3 + j];
                v += x * y;
            }
            c[i * 3 + j] = v;
        }
}

/* product of four links W1 W2 W3 W4, each with its own dagger flag */
static void m3_loop(const cplx *w[4], const int d[4], cplx *out)
{
    cplx t1[9], t2[9];
    m3_mul(w[0], d[0], w[1], d[1], t1);
    m3_mul(t1, 0, w[2], d[2], t2);
    m3_mul(t2, 0, w[3], d[3], out);
}

/* site index of c + a m + b n with periodic wrap */
static long shifted(const lattice *g, const int c[4], int m, int a, int n, int b)
{
    int y[4] = {c[0], c[1], c[2], c[3]};
    y[m] = ((y[m] + a) % g->L[m] + g->L[m]) % g->L[m];
    y[n] = ((y[n] + b) % g->L[n] + g->L[n]) % g->L[n];
    return site_index(g, y);
}

static void field_strength(const lattice *g, const cplx *U, long s, int m, int n, cplx F[9])
{
    int c[4];
    site_coords(g, s, c);
#define LK(site, dir) (U + ((site) * 4 + (dir)) * 9)
    const long xm = shifted(g, c, m, 1, n, 0), xn = shifted(g, c, m, 0, n, 1);
    const long xmm = shifted(g, c, m, -1, n, 0), xnm = shifted(g, c, m, 0, n, -1);
    const long xmm_np = shifted(g, c, m, -1, n, 1), xmm_nm = shifted(g, c, m, -1, n, -1);
    const long xmp_nm = shifted(g, c, m, 1, n, -1);
    cplx Q[9] = {0}, leaf[9];
    /* x -> x+m -> x+m+n -> x+n -> x */
    const cplx *w1[4] = {LK(s, m), LK(xm, n), LK(xn, m), LK(s, n)};
    const int d1[4] = {0, 0, 1, 1};
    /* x -> x+n -> x+n-m -> x-m -> x */
    const cplx *w2[4] = {LK(s, n), LK(xmm_np, m), LK(xmm, n), LK(xmm, m)};
    const int d2[4] = {0, 1, 1, 0};
    /* x -> x-m -> x-m-n -> x-n -> x */
    const cplx *w3[4] = {LK(xmm, m), LK(xmm_nm, n), LK(xmm_nm, m), LK(xnm, n)};
    const int d3[4] = {1, 1, 0, 0};
    /* x -> x-n -> x-n+m -> x+m -> x */
    const cplx *w4[4] = {LK(xnm, n), LK(xnm, m), LK(xmp_nm, n), LK(s, m)};
    const int d4[4] = {1, 0, 0, 1};
#undef LK
    const cplx **ws[4] = {w1, w2, w3, w4};
    const int *ds[4] = {d1, d2, d3, d4};
    for (int l = 0; l < 4; ++l) {
        m3_loop(ws[l], ds[l], leaf);
        for (int k = 0; k < 9; ++k) Q[k] += leaf[k];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / 8.0;
}

/* A(x) for every site: A_ out[V][12][12] complex */
void or_clover(const int32_t *L, const double *U_, double kappa, double csw, double *A_)
{
    lattice g = make_lattice(L, 0);
    const cplx *U = (const cplx *)U_;
    cplx *A = (cplx *)A_;
    cplx gm[4][4][4], sig[4][4][4][4];
    for (int mu = 0; mu < 4; ++mu) gamma_matrix(mu, gm[mu]);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx v = 0;
                    for (int k = 0; k < 4; ++k) v += gm[m][i][k] * gm[n][k][j] - gm[n][i][k] * gm[m][k][j];
                    sig[m][n][i][j] = 0.5 * I * v;
                }
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        cplx *a = A + s * 144;
        for (int k = 0; k < 144; ++k) a[k] = 0;
        for (int k = 0; k < 12; ++k) a[k * 12 + k] = 1;
        for (int m = 0; m < 4; ++m)
            for (int n = m + 1; n < 4; ++n) {
                cplx F[9];
                field_strength(&g, U, s, m, n, F);
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j)
                        for (int aa = 0; aa < 3; ++aa)
                            for (int bb = 0; bb < 3; ++bb)
                                a[(i * 3 + aa) * 12 + j * 3 + bb] += I * kappa * csw * sig[m][n][i][j] * F[aa * 3 + bb];
            }
    }
}

/* inverse of a 12 x 12 complex matrix by Gauss-Jordan elimination with
 * partial pivoting; returns 0 on success */
static int inv12(const cplx *a, cplx *out)
{
    cplx m[12][24];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 24; ++j) m[i][j] = j < 12 ? a[i * 12 + j] : (j - 12 == i ? 1.0 : 0.0);
    for (int col = 0; col < 12; ++col) {
        int piv = col;
        for (int r = col + 1; r < 12; ++r)
            if (cabs(m[r][col]) > cabs(m[piv][col])) piv = r;
        if (cabs(m[piv][col]) == 0.0) return 1;
        if (piv != col)
            for (int j = 0; j < 24; ++j) {
                cplx t = m[col][j];
                m[col][j] = m[piv][j];
                m[piv][j] = t;
            }
        cplx d = m[col][col];
        for (int j = 0; j < 24; ++j) m[col][j] /= d;
        for (int r = 0; r < 12; ++r)
            if (r != col && m[r][col] != 0) {
                cplx f = m[r][col];
                for (int j = 0; j < 24; ++j) m[r][j] -= f * m[col][j];
            }
    }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) out[i * 12 + j] = m[i][j + 12];
    return 0;
}

/* out_s = M_s in_s at the sites of the given parity (-1: all); other sites 0 */
static void apply_site_matrix(const lattice *g, const cplx *M, const cplx *in, cplx *out, int parity)
{
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g->V; ++s) {
        int c[4];
        site_coords(g, s, c);
        if (parity >= 0 && site_parity(c) != parity) {
            for (int k = 0; k < 12; ++k) out[s * 12 + k] = 0;
            continue;
        }
        for (int i = 0; i < 12; ++i) {
            cplx v = 0;
            for (int j = 0; j < 12; ++j) v += M[s * 144 + i * 12 + j] * in[s * 12 + j];
            out[s * 12 + i] = v;
        }
    }
}

/* out = D_k in = A in - kappa H in (dagger: A in - kappa H^dagger in), whole lattice */
void or_wilson_clover(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *in_,
                      double *out_, int32_t nrhs, double kappa, double csw, int32_t dagger)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long n = g.V * 12;
    cplx *A = malloc(sizeof(cplx) * 144 * g.V), *t = malloc(sizeof(cplx) * n);
    or_clover(L, U, kappa, csw, (double *)A);
    or_hop(L, antiperiodic_t, U, in_, out_, nrhs, -1, dagger);
    for (int r = 0; r < nrhs; ++r) {
        const cplx *in = (const cplx *)in_ + (size_t)r * n;
        cplx *out = (cplx *)out_ + (size_t)r * n;
        apply_site_matrix(&g, A, in, t, -1);
        vaxpby(1.0, t, -kappa, out, n);
    }
    free(A); free(t);
}

/* Even-odd CGNR for the clover operator, on the asymmetric Schur complement
 *   M = A_ee - kappa^2 D_eo A_oo^{-1} D_oe,  M^dagger = A_ee - kappa^2 D_oe^dagger A_oo^{-1} D_eo^dagger
 *   b' = eta_e + kappa D_eo A_oo^{-1} eta_o;   psi_o = A_oo^{-1} (eta_o + kappa D_oe psi_e)
 * with the same recurrence, stop test and outputs as or_cg_eo. */
int32_t or_cg_eo_clover(const int32_t *L, int32_t antiperiodic_t, const double *U, const double *eta_,
                        double *x_, int32_t nrhs, double kappa, double csw, double tol, int32_t maxiter,
                        int32_t *iters_out, double *resid_out)
{
    lattice g = make_lattice(L, antiperiodic_t);
    long V = g.V, n = V * 12;
    cplx *A = malloc(sizeof(cplx) * 144 * V), *Ai = malloc(sizeof(cplx) * 144 * V);
    cplx *bp = malloc(sizeof(cplx) * n), *rt = malloc(sizeof(cplx) * n);
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *t1 = malloc(sizeof(cplx) * n), *t2 = malloc(sizeof(cplx) * n);
    int32_t status = 0;
    or_clover(L, U, kappa, csw, (double *)A);
    for (long s = 0; s < V; ++s)
        if (inv12(A + s * 144, Ai + s * 144)) status = 1;
    /* out = M in (dagger: M^dagger in) on even-site vectors */
#define CLOV_SCHUR(in, out, dag)                                                                  \
    do {                                                                                          \
        or_hop(L, antiperiodic_t, U, (const double *)(in), (double *)t1, 1, 1, (dag));           \
        apply_site_matrix(&g, Ai, t1, t2, 1);                                                     \
        or_hop(L, antiperiodic_t, U, (const double *)t2, (double *)(out), 1, 0, (dag));          \
        apply_site_matrix(&g, A, (in), t1, 0);                                                    \
        vaxpby(1.0, t1, -kappa * kappa, (out), n);                                                \
    } while (0)

    for (int rh = 0; rh < nrhs && status == 0; ++rh) {
        const cplx *eta = (const cplx *)eta_ + (size_t)rh * n;
        cplx *x = (cplx *)x_ + (size_t)rh * n;
        double eta_norm = sqrt(vnorm2(eta, n));
        int it = 0, converged = 0;
        /* b' = eta_e + kappa D_eo A_oo^{-1} eta_o */
        apply_site_matrix(&g, Ai, eta, t1, 1);
        or_hop(L, antiperiodic_t, U, (const double *)t1, (double *)bp, 1, 0, 0);
        vaxpby(1.0, eta, kappa, bp, n);
        vzero_parity(&g, bp, 1);
        vzero_parity(&g, x, 1);
        if (eta_norm == 0.0) {
            memset(x, 0, sizeof(cplx) * n);
            iters_out[rh] = 0;
            resid_out[rh] = 0.0;
            continue;
        }
        CLOV_SCHUR(x, q, 0);
        memcpy(rt, bp, sizeof(cplx) * n);
        vaxpby(-1.0, q, 1.0, rt, n);
        CLOV_SCHUR(rt, r, 1);
        memcpy(p, r, sizeof(cplx) * n);
        double gam = vnorm2(r, n);
        while (it < maxiter) {
            if (sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
                CLOV_SCHUR(x, q, 0);
                memcpy(rt, bp, sizeof(cplx) * n);
                vaxpby(-1.0, q, 1.0, rt, n);
                if (sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
                    converged = 1;
                    break;
                }
                CLOV_SCHUR(rt, r, 1);
                gam = vnorm2(r, n);
                memcpy(p, r, sizeof(cplx) * n);
            }
            CLOV_SCHUR(p, q, 0);
            double alpha = gam / vnorm2(q, n);
            vaxpby(alpha, p, 1.0, x, n);
            vaxpby(-alpha, q, 1.0, rt, n);
            CLOV_SCHUR(rt, r, 1);
            double gam_new = vnorm2(r, n);
            vaxpby(1.0, r, gam_new / gam, p, n);
            gam = gam_new;
            ++it;
        }
        if (!converged && sqrt(vnorm2(rt, n)) <= tol * eta_norm) {
            CLOV_SCHUR(x, q, 0);
            memcpy(rt, bp, sizeof(cplx) * n);
            vaxpby(-1.0, q, 1.0, rt, n);
            converged = sqrt(vnorm2(rt, n)) <= tol * eta_norm;
        }
        /* psi_o = A_oo^{-1} (eta_o + kappa D_oe psi_e) */
        or_hop(L, antiperiodic_t, U, (const double *)x, (double *)t1, 1, 1, 0);
        vaxpby(1.0, eta, kappa, t1, n);
        apply_site_matrix(&g, Ai, t1, t2, 1);
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; ++s) {
            int c[4];
            site_coords(&g, s, c);
            if (site_parity(c) == 1)
                for (int k = 0; k < 12; ++k) x[s * 12 + k] = t2[s * 12 + k];
        }
        /* independent true residual with the whole-lattice operator */
        or_wilson_clover(L, antiperiodic_t, U, (const double *)x, (double *)t1, 1, kappa, csw, 0);
        vaxpby(1.0, eta, -1.0, t1, n);
        iters_out[rh] = it;
        resid_out[rh] = sqrt(vnorm2(t1, n)) / eta_norm;
        if (!converged) status = 1;
    }
#undef CLOV_SCHUR
    free(A); free(Ai); free(bp); free(rt); free(r); free(p); free(q); free(t1); free(t2);
    return status;
}

/* Number of OpenMP threads the oracle runs on. */
int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
