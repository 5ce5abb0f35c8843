"""GPU low-mode eigensolver of H_W and the deflated sign function / overlap
operator, through the C ABI, against dense eigendecomposition and the oracle."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests import dense_wilson as dw
from tests.gpu_util import from_dev, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu

RHO = 1.5


def dense_hw(L, U):
    kappa = 1.0 / (8 - 2 * RHO)
    V = li.volume(L)
    D = np.eye(12 * V) - kappa * dw.hopping_matrix(L, U)
    return dw.gamma5_matrix(V) @ D / (2 * kappa)


@pytest.fixture(scope="module")
def small():
    L = (4, 2, 2, 4)
    U = li.near_identity_links(L, 0.2, 1401)
    w, vec = np.linalg.eigh(dense_hw(L, U))
    return L, U, w, vec


def test_hw_eigs_match_dense(small):
    w_ = need_gpu()
    L, U, w, vec = small
    nev = 8
    V = li.volume(L)
    scale = 1.02 * (w ** 2).max()
    g = w_.Gauge(L, to_dev(U))
    ev = to_dev(np.zeros((nev, V, 4, 3), dtype=complex))
    st, lam, res, it = w_.wl_hw_eigs(g, RHO, nev, 16, 16, 1e-9, 300, scale, ev)
    got = from_dev(ev, (nev, V, 4, 3))
    want = w[np.argsort(np.abs(w))[:nev]]
    assert np.allclose(lam, want, rtol=0, atol=1e-10), (lam, want)
    assert max(res) <= 1e-9
    # the vectors are eigenvectors of the oracle's H_W and orthonormal
    for i in range(nev):
        hx = oracle.overlap_kernel(L, U, got[i], RHO)
        assert rel(hx, lam[i] * got[i]) <= 1e-8
    G = np.array([[np.vdot(got[i].ravel(), got[j].ravel()) for j in range(nev)] for i in range(nev)])
    assert np.abs(G - np.eye(nev)).max() <= 1e-12
    g.close()


@pytest.mark.parametrize("prec,gate", [("f64", 1e-12), ("f32", 1e-5)])
def test_deflated_sign_matches_oracle(small, prec, gate):
    """the same dense eigenpairs on both sides: the window leaves them out"""
    w_ = need_gpu()
    L, U, w, vec = small
    V = li.volume(L)
    nev = 32
    order = np.argsort(np.abs(w))
    xi = vec[:, order[:nev]].T.reshape(nev, V, 4, 3).copy()
    lam = w[order[:nev]]
    scale = 1.02 * (w ** 2).max()
    lo = 0.9 * w[order[nev]] ** 2 / scale
    psi = li.gaussian_spinor(L, 2401, nrhs=3)
    ref = oracle.sign_cheb_defl(L, U, psi, RHO, 200, lo, 1.0, scale, xi, lam)
    g = w_.Gauge(L, to_dev(U))
    out = to_dev(np.zeros_like(psi))
    w_.overlap_sign_cheb(g, to_dev(psi), out, 3, RHO, 200, lo, 1.0, scale, prec, 12, evecs=to_dev(xi), evals=lam)
    got = from_dev(out, psi.shape)
    for r in range(3):
        assert rel(got[r], ref[r]) <= gate, (r, rel(got[r], ref[r]))
    # and the deflated overlap operator, both orientations
    for dagger in (0, 1):
        refd = oracle.overlap(L, U, psi, RHO, 0.1, 200, lo, 1.0, scale, dagger=bool(dagger), evecs=xi, evals=lam)
        w_.overlap_dslash(g, to_dev(psi), out, 3, RHO, 0.1, 200, lo, 1.0, scale, dagger, prec, 12, evecs=to_dev(xi),
                          evals=lam)
        gotd = from_dev(out, psi.shape)
        for r in range(3):
            assert rel(gotd[r], refd[r]) <= gate, (dagger, r, rel(gotd[r], refd[r]))
    g.close()


def test_deflated_overlap_cg_with_gpu_eigenvectors():
    """6 x 4 x 4 x 6: GPU low modes deflate the sign of the overlap solve; the
    oracle's operator with the same modes confirms the residual."""
    w_ = need_gpu()
    L = (6, 4, 4, 6)
    U = li.near_identity_links(L, 0.2, 1402)
    V = li.volume(L)
    nev = 12
    v0 = li.gaussian_spinor(L, 7)
    scale = 1.02 * oracle.hw2_lmax(L, U, RHO, v0[0], iters=300)
    g = w_.Gauge(L, to_dev(U))
    ev = to_dev(np.zeros((nev, V, 4, 3), dtype=complex))
    st, lam, res, it = w_.wl_hw_eigs(g, RHO, nev, 20, 16, 1e-10, 300, scale, ev)
    assert max(res) <= 1e-10
    xi = from_dev(ev, (nev, V, 4, 3))
    lo = 0.9 * max(abs(x) for x in lam) ** 2 / scale
    eta = li.gaussian_spinor(L, 2402, nrhs=2)
    x = to_dev(np.zeros_like(eta))
    st, info = w_.overlap_cg(g, to_dev(eta), x, 2, RHO, 0.2, 200, lo, 1.0, scale, 1e-10, 3000, "f32", 12, 1e-3,
                             evecs=ev, evals=lam)
    got = from_dev(x, eta.shape)
    for r in range(2):
        assert info[r]["converged"] == 1 and info[r]["true_resid"] <= 1e-10, info[r]
        resid = rel(oracle.overlap(L, U, got[r], RHO, 0.2, 200, lo, 1.0, scale, evecs=xi, evals=lam), eta[r])
        assert resid <= 1.5e-10, (r, resid)
    g.close()
