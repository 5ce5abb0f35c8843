"""Pins of the oracle's clover term and clover solve (CPU only).

The clover (Sheikholeslami-Wohlert) operator D = A - kappa H with
A(x) = 1 + i kappa c_sw sum_{m<n} s_mn F_mn(x) is QUDA_DIRAC_CLOVER of the
paper's Table 1.  What fixes it independently of the oracle's code:
  * free field: F = 0, so A = 1 and D is the Wilson operator;
  * abelian constant field: U(1) links with flux B per plaquette in one plane
    (and B2 in another, on a commuting embedding) have every clover leaf equal
    to the plaquette, so F_mn = i sin(B) diag(1, -1, 0) exactly and
    A = 1 - kappa c_sw [sin B s_xy (x) diag(1,-1,0) + sin B2 s_zt (x) diag(0,1,-1)];
  * A is Hermitian and commutes with g5; D is g5-Hermitian and gauge covariant;
  * the even-odd CG solution matches a LAPACK solve of the dense operator.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests import dense_wilson as dw


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def sigma(m, n):
    g = dw.GAMMAS
    return 0.5j * (g[m] @ g[n] - g[n] @ g[m])


def flux_links(L, n1, n2):
    """Links with n1 flux quanta through the x-y plane (embedding diag(e^{ia}, e^{-ia}, 1))
    and n2 through the z-t plane (embedding diag(1, e^{ib}, e^{-ib})); returns (U, B1, B2)."""
    Lx, Ly, Lz, Lt = L
    B1 = 2 * np.pi * n1 / (Lx * Ly)
    B2 = 2 * np.pi * n2 / (Lz * Lt)
    c = dw.coords(L)
    V = len(c)
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    for s, (x, y, z, t) in enumerate(c):
        ph = np.zeros((4, 2))  # phase of embedding 1 (xy) and 2 (zt) per direction
        ph[0, 0] = -B1 * y
        if y == Ly - 1:
            ph[1, 0] = B1 * Ly * x
        ph[2, 1] = -B2 * t
        if t == Lt - 1:
            ph[3, 1] = B2 * Lt * z
        for mu in range(4):
            a, b = ph[mu]
            U[s, mu] = np.diag([np.exp(1j * a), np.exp(-1j * a + 1j * b), np.exp(-1j * b)])
    return U, B1, B2


def test_free_field_clover_is_identity():
    L = (4, 2, 2, 4)
    U = li.unit_links(L)
    A = oracle.clover(L, U, 0.12, 1.7)
    assert np.array_equal(A, np.broadcast_to(np.eye(12), A.shape))
    psi = li.gaussian_spinor(L, 3)
    assert rel(oracle.wilson_clover(L, U, psi, 0.12, 1.7), oracle.wilson(L, U, psi, 0.12)) < 1e-15


@pytest.mark.parametrize("n1,n2", [(1, 0), (0, 1), (1, 2)])
def test_abelian_flux_closed_form(n1, n2):
    L = (4, 6, 4, 6)
    U, B1, B2 = flux_links(L, n1, n2)
    kappa, csw = 0.11, 1.3
    A = oracle.clover(L, U, kappa, csw)
    want = np.eye(12) - kappa * csw * (np.sin(B1) * np.kron(sigma(0, 1), np.diag([1.0, -1.0, 0.0]))
                                       + np.sin(B2) * np.kron(sigma(2, 3), np.diag([0.0, 1.0, -1.0])))
    assert np.abs(A - want[None]).max() < 1e-14


@pytest.fixture(scope="module")
def rough():
    L = (4, 2, 2, 4)
    return L, li.haar_links(L, 41)


def test_clover_hermitian_chiral_blocks(rough):
    L, U = rough
    A = oracle.clover(L, U, 0.12, 1.9)
    assert np.abs(A - np.conj(np.swapaxes(A, 1, 2))).max() < 1e-15
    G5 = np.kron(dw.G5, np.eye(3))
    assert np.abs(G5 @ A - A @ G5).max() < 1e-15
    assert np.abs(A - np.eye(12)).max() > 0.05  # a rough field gives a sizeable term


def test_clover_gamma5_hermiticity_and_gauge_covariance(rough):
    L, U = rough
    kappa, csw = 0.12, 1.9
    phi = li.gaussian_spinor(L, 5)
    psi = li.gaussian_spinor(L, 6)
    Dpsi = oracle.wilson_clover(L, U, psi, kappa, csw)
    a = np.vdot(phi.ravel(), Dpsi.ravel())
    b = np.vdot(oracle.wilson_clover(L, U, phi, kappa, csw, dagger=True).ravel(), psi.ravel())
    assert abs(a - b) / abs(a) < 1e-13
    g5 = lambda v: v * np.array([1, 1, -1, -1])[None, :, None]
    assert rel(oracle.wilson_clover(L, U, psi, kappa, csw, dagger=True),
               g5(oracle.wilson_clover(L, U, g5(psi), kappa, csw))) < 1e-13
    # gauge covariance: D[U^W](W psi) = W D[U] psi
    V = li.volume(L)
    rng = np.random.default_rng(77)
    W = li.haar_su3_matrices(rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3)))
    c = dw.coords(L)
    Ug = np.empty_like(U)
    for s, x in enumerate(c):
        for mu in range(4):
            y = x.copy()
            y[mu] = (y[mu] + 1) % L[mu]
            Ug[s, mu] = W[s] @ U[s, mu] @ W[dw.index(L, y)].conj().T
    psi = psi[0]
    Dpsi = Dpsi[0]
    Wpsi = np.einsum("sab,sib->sia", W, psi)
    lhs = oracle.wilson_clover(L, Ug, Wpsi, kappa, csw)
    rhs = np.einsum("sab,sib->sia", W, Dpsi)
    assert rel(lhs, rhs) < 1e-13


@pytest.mark.parametrize("L,seed", [((2, 2, 2, 2), 43), ((4, 2, 2, 4), 44)])
def test_clover_cg_matches_dense_solve(L, seed):
    U = li.near_identity_links(L, 0.4, seed)
    kappa, csw = 0.12, 1.6
    V = li.volume(L)
    A = oracle.clover(L, U, kappa, csw)
    D = -kappa * dw.hopping_matrix(L, U)
    for s in range(V):
        D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += A[s]
    eta = li.gaussian_spinor(L, seed + 1000, nrhs=2)
    x, conv, iters, res = oracle.cg_eo_clover(L, U, eta, kappa, csw, tol=1e-12, maxiter=2000)
    assert conv and np.all(res <= 1e-12)
    for r in range(2):
        ref = np.linalg.solve(D, eta[r].ravel())
        assert rel(x[r], ref) < 1e-10
    # the whole-lattice operator of the oracle is the dense one
    assert rel(oracle.wilson_clover(L, U, eta[0], kappa, csw), D @ eta[0].ravel()) < 1e-14
