"""GPU solves of the Wilson system (even-odd CGNR, mixed precision with FP64
reliable updates, batched) through the C ABI, checked against the FP64 oracle.

For every solve the true residual |eta - D psi| / |eta| is recomputed by the
oracle's whole-lattice operator from the GPU solution (independent of the
GPU's own report), and the solution is compared with the oracle's solution:
|psi - psi_oracle| / |psi_oracle| <= 2 cond(D) tol.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import from_dev, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu


def true_resid(L, U, eta, psi, kappa):
    r = eta - oracle.wilson(L, U, psi, kappa)
    return np.linalg.norm(r.reshape(r.shape[0], -1), axis=1) / np.linalg.norm(eta.reshape(eta.shape[0], -1), axis=1)


def solve(w, L, U, eta, kappa, tol, sloppy, recon=12, delta=0.1, maxiter=2000, check=True, x0=None):
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta) if x0 is None else x0)
    st, info = w.wilson_cg(g, to_dev(eta), x, eta.shape[0], kappa, tol, maxiter, sloppy, recon, delta, check=check)
    out = from_dev(x, eta.shape)
    g.close()
    return st, info, out


def test_config1_plain_fp64_4x4():
    """4^4 Haar links, kappa 0.12, Gaussian source, FP64 throughout, tol 1e-12."""
    w = need_gpu()
    L = (4, 4, 4, 4)
    U = li.haar_links(L, 1001)
    eta = li.gaussian_spinor(L, 2001)
    st, info, x = solve(w, L, U, eta, 0.12, 1e-12, "f64", 18)
    ref, conv, it, _ = oracle.cg_eo(L, U, eta, 0.12, 1e-12)
    tr = true_resid(L, U, eta, x, 0.12)
    assert info[0]["converged"] and tr[0] <= 1e-12
    assert abs(info[0]["true_resid"] - tr[0]) <= 1e-13
    assert rel(x, ref) <= 2 * 4.0 * 1e-12  # cond(D) = 3.96 for this configuration
    assert abs(info[0]["iters"] - it[0]) <= 6


@pytest.mark.parametrize("sloppy,recon", [("f32", 12), ("f32", 18), ("f16", 12), ("bf16", 12), ("f64", 12)])
def test_mixed_precision_reaches_1e10(sloppy, recon):
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2002, nrhs=2)
    st, info, x = solve(w, L, U, eta, 0.1245, 1e-10, sloppy, recon)
    tr = true_resid(L, U, eta, x, 0.1245)
    ref, _, _, _ = oracle.cg_eo(L, U, eta, 0.1245, 1e-12)
    for r in range(2):
        assert info[r]["converged"] and tr[r] <= 1e-10, (sloppy, info[r], tr[r])
        assert abs(info[r]["true_resid"] - tr[r]) <= 1e-3 * tr[r] + 1e-15
        assert info[r]["reliable_updates"] >= 1
    assert rel(x, ref) <= 2 * 20 * 1e-10


def test_point_sources_twelve_rhs():
    """The 12 spin-colour point sources at the origin, solved together."""
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1004)
    eta = li.point_sources(L)
    st, info, x = solve(w, L, U, eta, 0.1245, 1e-10, "f32")
    tr = true_resid(L, U, eta, x, 0.1245)
    assert np.all(tr <= 1e-10) and all(i["converged"] for i in info)
    # the solution of one source alone agrees with the batched one
    st1, info1, x1 = solve(w, L, U, eta[5:6], 0.1245, 1e-10, "f32")
    assert rel(x1[0], x[5]) <= 1e-9


def test_uneven_batch_multi():
    """Lattices of different sizes, kappas and RHS counts in one batched solve."""
    w = need_gpu()
    specs = [((4, 4, 4, 4), 0.12, 2), ((6, 6, 6, 6), 0.1245, 1), ((4, 4, 4, 8), 0.124, 3), ((8, 8, 8, 4), 0.1245, 1)]
    gs, etas, xs, Us = [], [], [], []
    for i, (L, k, n) in enumerate(specs):
        U = li.near_identity_links(L, 0.3, 3000 + i)
        Us.append(U)
        gs.append(w.Gauge(L, to_dev(U)))
        e = li.gaussian_spinor(L, 4000 + i, nrhs=n)
        etas.append(e)
        xs.append(to_dev(np.zeros_like(e)))
    st, info = w.wilson_cg_multi(gs, [to_dev(e) for e in etas], xs, [s[2] for s in specs], [s[1] for s in specs],
                                 1e-10, 2000, "f32", 12, 0.1)
    j = 0
    for i, (L, k, n) in enumerate(specs):
        x = from_dev(xs[i], etas[i].shape)
        tr = true_resid(L, Us[i], etas[i], x, k)
        assert np.all(tr <= 1e-10), (i, tr)
        for r in range(n):
            assert info[j]["converged"]
            j += 1
    for g in gs:
        g.close()


def test_solver_edge_cases():
    w = need_gpu()
    L = (4, 4, 4, 4)
    U = li.haar_links(L, 1001)
    eta = li.gaussian_spinor(L, 2001, nrhs=2)
    eta[1] = 0.0  # a zero source gives x = 0, converged
    st, info, x = solve(w, L, U, eta, 0.12, 1e-10, "f32", x0=np.ones_like(eta))
    assert info[1]["converged"] and info[1]["iters"] == 0 and np.abs(x[1]).max() == 0.0
    assert info[0]["converged"]
    # a converged guess needs no iterations
    st, info2, x2 = solve(w, L, U, eta[:1], 0.12, 1e-10, "f32", x0=x[:1])
    assert info2[0]["converged"] and info2[0]["iters"] == 0
    # maxiter too small: NOCONV with info filled and the iterate returned
    st, info3, x3 = solve(w, L, U, eta[:1], 0.12, 1e-12, "f32", maxiter=2, check=False)
    assert st == w.WL_ERR_NOCONV and info3[0]["converged"] == 0 and info3[0]["iters"] >= 2
    assert 0 < info3[0]["true_resid"] < 1
    # a NaN in the source is reported, not iterated
    bad = eta[:1].copy()
    bad[0, 7, 1, 2] = np.nan
    st, info4, _ = solve(w, L, U, bad, 0.12, 1e-10, "f32", check=False)
    assert st == w.WL_ERR_NONFINITE
    # invalid arguments
    g = w.Gauge(L, to_dev(U))
    d = to_dev(eta[:1])
    for args in [(1, -0.1, 1e-10, 10), (1, 0.12, 0.0, 10), (1, 0.12, 1e-10, 0), (0, 0.12, 1e-10, 10)]:
        st, _ = w.wilson_cg(g, d, to_dev(eta[:1]), *args, check=False)
        assert st == w.WL_ERR_ARG
    st, _ = w.wilson_cg(g, d, to_dev(eta[:1]), 1, 0.12, 1e-10, 10, "f32", 12, 1.5, check=False)
    assert st == w.WL_ERR_ARG
    g.close()


def test_config2_size_fp32_and_fp64():
    """24^3 x 48, eps = 0.3, kappa = 0.1245, tol 1e-10: plain FP64 and mixed FP32."""
    w = need_gpu()
    L = (24, 24, 24, 48)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2002)
    res = {}
    for sloppy, recon in [("f64", 18), ("f32", 12), ("f16", 12)]:
        st, info, x = solve(w, L, U, eta, 0.1245, 1e-10, sloppy, recon, delta=0.1)
        tr = true_resid(L, U, eta, x, 0.1245)
        assert info[0]["converged"] and tr[0] <= 1e-10, (sloppy, info, tr)
        res[sloppy] = x
    assert rel(res["f32"], res["f64"]) <= 1e-8
    assert rel(res["f16"], res["f64"]) <= 1e-8


def test_repeated_solves_across_streams():
    """One gauge handle solving the same batch four times: twice on one stream,
    then on a second stream, then on the current stream.  The batch has a zero
    source (masked out from the start) and two sources that converge at
    different iterations, so the active mask changes within each solve and
    across calls; the library skips a mask upload only when the same mask was
    the last one enqueued on the same stream.  Every solution must meet the
    tolerance by the oracle's operator, and the reductions being
    deterministic, all four are bit-identical."""
    import torch

    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2005, nrhs=3)
    eta[1] = 0.0
    eta[2] *= 1e-3
    g = w.Gauge(L, to_dev(U))
    d = to_dev(eta)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for s in (s1, s1, s2, None):
        x = to_dev(np.zeros_like(eta))
        torch.cuda.synchronize()
        st, info = w.wilson_cg(g, d, x, 3, 0.1245, 1e-10, 2000, "f16", 12, 0.1, stream=s)
        torch.cuda.synchronize()
        xo = from_dev(x, eta.shape)
        assert all(i["converged"] for i in info), info
        assert info[1]["iters"] == 0 and np.abs(xo[1]).max() == 0.0
        tr = true_resid(L, U, eta[[0, 2]], xo[[0, 2]], 0.1245)
        assert tr.max() <= 1e-10, tr
        outs.append(xo)
    g.close()
    for xo in outs[1:]:
        assert np.array_equal(xo, outs[0])


def test_one_handle_two_kappas_with_graphs():
    """A handle solved at one kappa and then at another replays no iteration
    chunk captured for the first: the second solve takes the iterations and
    reaches the residual of a solve on a fresh handle, and its solution agrees
    with that one to round-off."""
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2002, nrhs=2)
    for sloppy, method in (("f16", w.wilson_cg), ("f32", w.wilson_bicgstab)):
        g = w.Gauge(L, to_dev(U))
        d = to_dev(eta)
        x = to_dev(np.zeros_like(eta))
        method(g, d, x, 2, 0.12, 1e-10, 2000, sloppy, 12, 0.1)
        x.zero_()
        _, info = method(g, d, x, 2, 0.1245, 1e-10, 2000, sloppy, 12, 0.1)
        xa = from_dev(x, eta.shape)
        g.close()
        g2 = w.Gauge(L, to_dev(U))
        x2 = to_dev(np.zeros_like(eta))
        _, info2 = method(g2, d, x2, 2, 0.1245, 1e-10, 2000, sloppy, 12, 0.1)
        xb = from_dev(x2, eta.shape)
        g2.close()
        tr = true_resid(L, U, eta, xa, 0.1245)
        assert tr.max() <= 1e-10, (sloppy, tr)
        for r in range(2):
            assert info[r]["iters"] == info2[r]["iters"], (sloppy, info, info2)
            assert info[r]["reliable_updates"] == info2[r]["reliable_updates"]
        assert rel(xa, xb) <= 1e-12, (sloppy, rel(xa, xb))


@pytest.mark.parametrize("method", ["cgnr", "bicgstab", "multi"])
def test_graph_replay_matches_eager(method, monkeypatch):
    """The iteration chunks replayed from captured graphs and the same chunks
    launched one kernel at a time (WL_GRAPHS=0) give bit-identical solutions,
    iteration counts and update schedules: the graph path adds no race."""
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2003, nrhs=3)
    eta[2] *= 1e-3  # converges at another iteration: the mask changes inside the solve

    def run():
        g = w.Gauge(L, to_dev(U))
        x = to_dev(np.zeros_like(eta))
        if method == "multi":
            L2 = (4, 4, 4, 8)
            U2 = li.near_identity_links(L2, 0.3, 3001)
            e2 = li.gaussian_spinor(L2, 4001, nrhs=2)
            g2 = w.Gauge(L2, to_dev(U2))
            x2 = to_dev(np.zeros_like(e2))
            _, info = w.wilson_cg_multi([g, g2], [to_dev(eta), to_dev(e2)], [x, x2], [3, 2], [0.1245, 0.124],
                                        1e-10, 2000, "f16", 12, 0.1)
            out = np.concatenate([from_dev(x, eta.shape).ravel(), from_dev(x2, e2.shape).ravel()])
            g2.close()
        else:
            fn = w.wilson_cg if method == "cgnr" else w.wilson_bicgstab
            _, info = fn(g, to_dev(eta), x, 3, 0.1245, 1e-10, 2000, "f16", 12, 0.1)
            out = from_dev(x, eta.shape)
        g.close()
        return out, [(i["iters"], i["reliable_updates"], i["converged"]) for i in info]

    monkeypatch.delenv("WL_GRAPHS", raising=False)
    xg, ig = run()
    monkeypatch.setenv("WL_GRAPHS", "0")
    xe, ie = run()
    assert ig == ie, (ig, ie)
    assert all(c for _, _, c in ig)
    assert np.array_equal(xg, xe)


@pytest.mark.parametrize("method", ["cgnr", "bicgstab"])
@pytest.mark.parametrize("sloppy", ["f32", "f16"])
def test_streamed_fields_match_plain(method, sloppy, monkeypatch):
    """The solver-iteration kernels read and write fields non-temporally when
    the set is large against the last-level cache; the hint changes where
    data is cached, never a value: forced on and forced off
    (WL_STREAM_FIELDS), a solve gives bit-identical solutions and schedules."""
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2004, nrhs=2)

    def run():
        g = w.Gauge(L, to_dev(U))
        x = to_dev(np.zeros_like(eta))
        fn = w.wilson_cg if method == "cgnr" else w.wilson_bicgstab
        _, info = fn(g, to_dev(eta), x, 2, 0.1245, 1e-10, 2000, sloppy, 12, 0.1)
        out = from_dev(x, eta.shape)
        g.close()
        return out, [(i["iters"], i["reliable_updates"], i["converged"]) for i in info]

    monkeypatch.setenv("WL_STREAM_FIELDS", "0")
    xp, ip = run()
    monkeypatch.setenv("WL_STREAM_FIELDS", "1")
    xs, is_ = run()
    assert ip == is_, (ip, is_)
    assert all(c for _, _, c in ip)
    assert np.array_equal(xp, xs)
    tr = true_resid(L, U, eta, xs, 0.1245)
    assert np.all(tr <= 1e-10), tr


@pytest.mark.parametrize("sloppy", ["bf16", "f16"])
def test_stagnation_raises_the_sloppy_precision(sloppy):
    """With delta = 0.9 a reliable update follows every 10% fall of the sloppy
    residual, so the FP64 residual cannot halve between two updates: the
    stagnation rule restarts the search direction, and a second stall in a row
    raises the sloppy storage (FP16/BF16 -> FP32 -> FP64), after folding the
    sloppy solution into the FP64 accumulator.  The solve must still reach the
    tolerance, confirmed by the oracle's operator, and agree with the oracle's
    solution."""
    w = need_gpu()
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2002)
    st, info, x = solve(w, L, U, eta, 0.1245, 1e-10, sloppy, 12, delta=0.9, maxiter=5000)
    assert info[0]["precision_escalations"] >= 1, info
    assert info[0]["converged"] == 1, info
    tr = true_resid(L, U, eta, x, 0.1245)
    assert tr[0] <= 1e-10, tr
    ref, _, _, _ = oracle.cg_eo(L, U, eta, 0.1245, 1e-12)
    assert rel(x, ref) <= 2 * 20 * 1e-10
