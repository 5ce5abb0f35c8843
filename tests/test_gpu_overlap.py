"""GPU overlap operator and overlap CG through the C ABI, against the FP64
oracle (same Chebyshev polynomial, same scale)."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import from_dev, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu

RHO = 1.5
DEG = 200
LO, HI = 0.003, 1.0
# 6 x 4 x 4 x 6: 288 sites per parity, a ragged tail for every block size
L = (6, 4, 4, 6)


@pytest.fixture(scope="module")
def case():
    U = li.near_identity_links(L, 0.2, 1205)
    v0 = li.gaussian_spinor(L, 7)
    scale = 1.02 * oracle.hw2_lmax(L, U, RHO, v0[0], iters=200)
    return U, scale


@pytest.mark.parametrize("prec,recon,gate", [("f64", 18, 1e-12), ("f64", 12, 1e-12), ("f32", 12, 1e-5)])
@pytest.mark.parametrize("dagger", [0, 1])
def test_overlap_dslash_matches_oracle(case, prec, recon, gate, dagger):
    w = need_gpu()
    U, scale = case
    mass = 0.2
    psi = li.gaussian_spinor(L, 2201, nrhs=3)
    ref = oracle.overlap(L, U, psi, RHO, mass, DEG, LO, HI, scale, dagger=bool(dagger))
    g = w.Gauge(L, to_dev(U))
    out = to_dev(np.zeros_like(psi))
    w.overlap_dslash(g, to_dev(psi), out, 3, RHO, mass, DEG, LO, HI, scale, dagger, prec, recon)
    got = from_dev(out, psi.shape)
    for r in range(3):
        assert rel(got[r], ref[r]) <= gate, (r, rel(got[r], ref[r]))
    g.close()


@pytest.mark.parametrize("sloppy,delta", [("f64", 0.1), ("f32", 1e-3)])
def test_overlap_cg_matches_oracle(case, sloppy, delta):
    w = need_gpu()
    U, scale = case
    mass = 0.2
    tol = 1e-10
    eta = li.gaussian_spinor(L, 2202, nrhs=2)
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.overlap_cg(g, to_dev(eta), x, 2, RHO, mass, DEG, LO, HI, scale, tol, 2000, sloppy, 12, delta)
    got = from_dev(x, eta.shape)
    for r in range(2):
        assert info[r]["converged"] == 1 and info[r]["true_resid"] <= tol, info[r]
        # the oracle's operator confirms the residual of the GPU solution
        res = rel(oracle.overlap(L, U, got[r], RHO, mass, DEG, LO, HI, scale), eta[r])
        assert res <= 1.5 * tol, (r, res)
    # and the solution agrees with the oracle's own solve (cond(D) <= 2 rho / m)
    ref, conv, iters, resid = oracle.overlap_cg(L, U, eta[0], RHO, mass, DEG, LO, HI, scale, tol=1e-11)
    assert conv
    assert rel(got[0], ref) <= (2 * RHO / mass) * 2e-10
    g.close()


def test_overlap_cg_zero_source_and_validation(case):
    w = need_gpu()
    U, scale = case
    eta = li.gaussian_spinor(L, 2203, nrhs=2)
    eta[1] = 0
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.ones_like(eta))
    st, info = w.overlap_cg(g, to_dev(eta), x, 2, RHO, 0.3, DEG, LO, HI, scale, 1e-9, 2000, "f64", 18, 0.1)
    got = from_dev(x, eta.shape)
    assert info[1]["converged"] == 1 and info[1]["iters"] == 0 and np.all(got[1] == 0)
    assert info[0]["converged"] == 1 and info[0]["true_resid"] <= 1e-9
    # mass 0 has exact zero modes: refused before any device work
    with pytest.raises(w.WilsonError) as e:
        w.overlap_cg(g, to_dev(eta), x, 2, RHO, 0.0, DEG, LO, HI, scale, 1e-9, 100, "f64", 18, 0.1)
    assert e.value.status == w.WL_ERR_ARG
    with pytest.raises(w.WilsonError) as e:
        w.overlap_dslash(g, to_dev(eta), x, 2, RHO, 0.1, DEG, LO, HI, scale, 0, "f16", 12)
    assert e.value.status == w.WL_ERR_PREC
    g.close()


def test_overlap_cg_single_rhs(case):
    """One right-hand side (the GWU-code inverter's usual call): both parities
    of each H_W application run in one launch inside every sign evaluation."""
    w = need_gpu()
    U, scale = case
    mass, tol = 0.2, 1e-10
    eta = li.gaussian_spinor(L, 2204)
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.overlap_cg(g, to_dev(eta), x, 1, RHO, mass, DEG, LO, HI, scale, tol, 2000, "f32", 12, 1e-3)
    got = from_dev(x, eta.shape)
    assert info[0]["converged"] == 1 and info[0]["true_resid"] <= tol, info[0]
    assert rel(oracle.overlap(L, U, got[0], RHO, mass, DEG, LO, HI, scale), eta[0]) <= 1.5 * tol
    g.close()
