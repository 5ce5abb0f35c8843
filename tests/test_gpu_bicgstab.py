"""GPU BiCGStab on the even-odd Schur system (mixed precision, FP64 reliable
updates) through the C ABI.  The solution of D psi = eta is unique, so it is
checked exactly as the CGNR solutions are: the oracle's whole-lattice operator
recomputes the true residual from the GPU solution, and the solution is
compared with the oracle's own solve."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import from_dev, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu


def true_resid(L, U, eta, psi, kappa):
    r = eta - oracle.wilson(L, U, psi, kappa)
    return np.linalg.norm(r.reshape(r.shape[0], -1), axis=1) / np.linalg.norm(eta.reshape(eta.shape[0], -1), axis=1)


def solve(w, L, U, eta, kappa, tol, sloppy, recon=12, delta=0.1, maxiter=3000, check=True):
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.wilson_bicgstab(g, to_dev(eta), x, eta.shape[0], kappa, tol, maxiter, sloppy, recon, delta,
                                 check=check)
    out = from_dev(x, eta.shape)
    g.close()
    return st, info, out


def test_bicgstab_fp64_4x4():
    w = need_gpu()
    L = (4, 4, 4, 4)
    U = li.haar_links(L, 1001)
    eta = li.gaussian_spinor(L, 2001)
    st, info, x = solve(w, L, U, eta, 0.12, 1e-12, "f64", 18)
    ref, _, _, _ = oracle.cg_eo(L, U, eta, 0.12, 1e-13)
    tr = true_resid(L, U, eta, x, 0.12)
    assert info[0]["converged"] and tr[0] <= 1e-12
    assert rel(x, ref) <= 2 * 4.0 * 1e-12


@pytest.mark.parametrize("sloppy", ["f32", "f16", "bf16"])
def test_bicgstab_mixed_8x4(sloppy):
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2002, nrhs=2)
    st, info, x = solve(w, L, U, eta, 0.1245, 1e-10, sloppy)
    tr = true_resid(L, U, eta, x, 0.1245)
    ref, _, _, _ = oracle.cg_eo(L, U, eta, 0.1245, 1e-12)
    for r in range(2):
        assert info[r]["converged"] and tr[r] <= 1e-10, (sloppy, info[r], tr[r])
        assert abs(info[r]["true_resid"] - tr[r]) <= 1e-3 * tr[r] + 1e-15
    assert rel(x, ref) <= 2 * 20 * 1e-10


def test_bicgstab_point_sources():
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1004)
    eta = li.point_sources(L)
    st, info, x = solve(w, L, U, eta, 0.1245, 1e-10, "f32")
    tr = true_resid(L, U, eta, x, 0.1245)
    assert np.all(tr <= 1e-10) and all(i["converged"] for i in info)


def test_bicgstab_24c48():
    w = need_gpu()
    L = (24, 24, 24, 48)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2002)
    for sloppy in ("f32", "f16"):
        st, info, x = solve(w, L, U, eta, 0.1245, 1e-10, sloppy)
        tr = true_resid(L, U, eta, x, 0.1245)
        assert info[0]["converged"] and tr[0] <= 1e-10, (sloppy, info, tr)


def test_bicgstab_edge_cases():
    w = need_gpu()
    L = (4, 4, 4, 4)
    U = li.haar_links(L, 1001)
    eta = li.gaussian_spinor(L, 2001, nrhs=2)
    eta[1] = 0.0
    st, info, x = solve(w, L, U, eta, 0.12, 1e-10, "f32")
    assert info[1]["converged"] and info[1]["iters"] == 0 and np.abs(x[1]).max() == 0.0
    assert info[0]["converged"]
    st, info, x = solve(w, L, U, eta[:1], 0.12, 1e-12, "f32", maxiter=2, check=False)
    assert st == w.WL_ERR_NOCONV and info[0]["converged"] == 0 and info[0]["iters"] >= 2
