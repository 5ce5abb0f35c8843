"""Pins of the oracle's overlap operator and its CG solve (CPU only).

The overlap operator D_ov(m) = (rho + m/2) + (rho - m/2) g5 eps(H_W) is the
operator GWU-code inverts (Sections 1 and 3).  Its properties with the exact
sign function are fixed by the mathematics, not by the oracle:
  * dense check: with a Chebyshev window that covers the spectrum of H_W^2,
    the oracle's D_ov matches a + b g5 V sign(L) V^dagger built from numpy
    eigh of an independently assembled dense H_W;
  * Ginsparg-Wilson relation at m = 0: g5 D + D g5 = D g5 D / rho;
  * g5 eps is unitary, so D(0)/rho - 1 preserves norms, and D is normal;
  * D(m) = (1 - m / (2 rho)) D(0) + m;
  * the CG solution matches a LAPACK solve of the dense exact operator;
  * deflation: with the lowest eigenvectors of H_W treated exactly, a window
    that leaves them out still gives the exact sign function, while the
    undeflated polynomial on that window does not.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests import dense_wilson as dw

RHO = 1.5
DEG = 200


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def g5(psi):
    out = np.array(psi, copy=True)
    out[..., 2:, :] *= -1
    return out


def make_case():
    L = (4, 2, 2, 4)
    U = li.near_identity_links(L, 0.2, 1105)
    kappa = 1.0 / (8 - 2 * RHO)
    V = li.volume(L)
    D = np.eye(12 * V) - kappa * dw.hopping_matrix(L, U)
    HW = dw.gamma5_matrix(V) @ D / (2 * kappa)
    w, vec = np.linalg.eigh(HW)
    lam2 = w ** 2
    scale = 1.02 * lam2.max()
    lo = 0.9 * lam2.min() / scale
    S = (vec * np.sign(w)) @ vec.conj().T
    G5 = dw.gamma5_matrix(V)
    return {"L": L, "U": U, "V": V, "scale": scale, "lo": lo, "S": S, "G5": G5, "w": w, "vec": vec}


@pytest.fixture(scope="module")
def ov():
    return make_case()


def apply(ov, psi, mass, dagger=False):
    return oracle.overlap(ov["L"], ov["U"], psi, RHO, mass, DEG, ov["lo"], 1.0, ov["scale"], dagger=dagger)


def dense_overlap(ov, mass):
    n = ov["S"].shape[0]
    return (RHO + 0.5 * mass) * np.eye(n) + (RHO - 0.5 * mass) * ov["G5"] @ ov["S"]


@pytest.mark.parametrize("mass", [0.0, 0.25])
def test_overlap_matches_dense_exact_sign(ov, mass):
    psi = li.gaussian_spinor(ov["L"], 2101, nrhs=2)
    Dd = dense_overlap(ov, mass)
    got = apply(ov, psi, mass)
    gotd = apply(ov, psi, mass, dagger=True)
    for r in range(2):
        assert rel(got[r], Dd @ psi[r].ravel()) < 1e-9
        assert rel(gotd[r], Dd.conj().T @ psi[r].ravel()) < 1e-9


def test_overlap_ginsparg_wilson_and_normality(ov):
    psi = li.gaussian_spinor(ov["L"], 2102)
    D0 = lambda v: apply(ov, v, 0.0)
    lhs = g5(D0(psi)) + D0(g5(psi))
    rhs = D0(g5(D0(psi))) / RHO
    assert rel(lhs, rhs) < 1e-9
    # g5 eps = D(0)/rho - 1 is unitary: norms are preserved
    u = D0(psi) / RHO - psi
    assert abs(np.linalg.norm(u) / np.linalg.norm(psi) - 1) < 1e-9
    # normal operator: |D psi| = |D^dagger psi|
    m = 0.3
    assert abs(np.linalg.norm(apply(ov, psi, m)) / np.linalg.norm(apply(ov, psi, m, dagger=True)) - 1) < 1e-9


def test_overlap_adjoint_and_mass_dependence(ov):
    phi = li.gaussian_spinor(ov["L"], 2103)
    psi = li.gaussian_spinor(ov["L"], 2104)
    m = 0.4
    a = np.vdot(phi.ravel(), apply(ov, psi, m).ravel())
    b = np.vdot(apply(ov, phi, m, dagger=True).ravel(), psi.ravel())
    assert abs(a - b) / abs(a) < 1e-12
    # D(m) = (1 - m / (2 rho)) D(0) + m
    lin = (1 - m / (2 * RHO)) * apply(ov, psi, 0.0) + m * psi
    assert rel(apply(ov, psi, m), lin) < 1e-12


def test_overlap_cg_matches_dense_solve(ov):
    mass = 0.2
    eta = li.gaussian_spinor(ov["L"], 2105, nrhs=2)
    x, conv, iters, res = oracle.overlap_cg(ov["L"], ov["U"], eta, RHO, mass, DEG, ov["lo"], 1.0, ov["scale"],
                                            tol=1e-11, maxiter=150)
    assert conv and np.all(res <= 1e-11)
    Dd = dense_overlap(ov, mass)
    for r in range(2):
        ref = np.linalg.solve(Dd, eta[r].ravel())
        assert rel(x[r], ref) < 1e-8
    assert np.all(iters > 0)


def test_overlap_cg_zero_source_and_guess(ov):
    mass = 0.2
    eta = li.gaussian_spinor(ov["L"], 2106)
    z, conv, iters, res = oracle.overlap_cg(ov["L"], ov["U"], np.zeros_like(eta), RHO, mass, DEG, ov["lo"], 1.0,
                                            ov["scale"], tol=1e-10)
    assert conv and np.all(z == 0) and iters[0] == 0
    x, conv, iters, res = oracle.overlap_cg(ov["L"], ov["U"], eta, RHO, mass, DEG, ov["lo"], 1.0, ov["scale"],
                                            tol=1e-10)
    # the converged solution as the initial guess needs no iteration
    x2, conv2, iters2, res2 = oracle.overlap_cg(ov["L"], ov["U"], eta, RHO, mass, DEG, ov["lo"], 1.0, ov["scale"],
                                               tol=1e-10, x0=x)
    assert conv and conv2 and iters2[0] == 0 and res2[0] <= 1e-10


def low_modes(ov, nev):
    """The nev eigenpairs of the dense H_W of smallest |lambda|, as canonical fields."""
    order = np.argsort(np.abs(ov["w"]))[:nev]
    vecs = ov["vec"][:, order].T.reshape(nev, ov["V"], 4, 3)
    return vecs, ov["w"][order], np.abs(ov["w"][np.argsort(np.abs(ov["w"]))[nev]])


def test_deflated_sign_is_exact_outside_the_window(ov):
    nev = 32
    vecs, lam, next_abs = low_modes(ov, nev)
    lo = 0.9 * next_abs ** 2 / ov["scale"]  # the window leaves out the deflated modes
    assert lo > 1.2 * ov["lo"]
    psi = li.gaussian_spinor(ov["L"], 2107, nrhs=2)
    got = oracle.sign_cheb_defl(ov["L"], ov["U"], psi, RHO, DEG, lo, 1.0, ov["scale"], vecs, lam)
    for r in range(2):
        assert rel(got[r], ov["S"] @ psi[r].ravel()) < 1e-9
    # without the deflation the same window misses the low modes
    plain = oracle.sign_cheb(ov["L"], ov["U"], psi, RHO, DEG, lo, 1.0, ov["scale"])
    assert rel(plain[0], ov["S"] @ psi[0].ravel()) > 1e-6
    # the deflated overlap operator satisfies Ginsparg-Wilson on that window too
    D0 = lambda v: oracle.overlap(ov["L"], ov["U"], v, RHO, 0.0, DEG, lo, 1.0, ov["scale"], evecs=vecs, evals=lam)
    lhs = g5(D0(psi[0])) + D0(g5(psi[0]))
    assert rel(lhs, D0(g5(D0(psi[0]))) / RHO) < 1e-9


def test_deflated_overlap_cg_matches_dense_solve(ov):
    nev = 32
    vecs, lam, next_abs = low_modes(ov, nev)
    lo = 0.9 * next_abs ** 2 / ov["scale"]
    mass = 0.2
    eta = li.gaussian_spinor(ov["L"], 2108)
    x, conv, iters, res = oracle.overlap_cg(ov["L"], ov["U"], eta, RHO, mass, DEG, lo, 1.0, ov["scale"], tol=1e-11,
                                            maxiter=150, evecs=vecs, evals=lam)
    assert conv and res[0] <= 1e-11
    assert rel(x, np.linalg.solve(dense_overlap(ov, mass), eta.ravel())) < 1e-8
