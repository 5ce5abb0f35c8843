"""GPU Wilson-clover operator and its even-odd solvers through the C ABI,
against the FP64 oracle (clover term built independently on both sides)."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import (from_dev, half_storage_excess, need_gpu, quantize_links, quantize_spinor, rel,
                            to_dev)

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.12, 1.6
# 6 x 4 x 4 x 6: 288 sites per parity, a ragged tail for every block size
L = (6, 4, 4, 6)


@pytest.fixture(scope="module")
def links():
    return li.near_identity_links(L, 0.4, 1301)


@pytest.mark.parametrize("prec,recon,gate", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 12, 1e-6),
                                             ("f32", 18, 1e-6)])
@pytest.mark.parametrize("dagger", [0, 1])
def test_clover_dslash_matches_oracle(links, prec, recon, gate, dagger):
    w = need_gpu()
    psi = li.gaussian_spinor(L, 2301, nrhs=2)
    ref = oracle.wilson_clover(L, links, psi, KAPPA, CSW, dagger=bool(dagger))
    g = w.Gauge(L, to_dev(links))
    out = to_dev(np.zeros_like(psi))
    w.wilson_clover_dslash(g, to_dev(psi), out, 2, KAPPA, CSW, dagger, prec, recon)
    got = from_dev(out, psi.shape)
    for r in range(2):
        assert rel(got[r], ref[r]) <= gate, (r, rel(got[r], ref[r]))
    # c_sw = 0 is the Wilson operator
    w.wilson_clover_dslash(g, to_dev(psi), out, 2, KAPPA, 0.0, dagger, prec, recon)
    assert rel(from_dev(out, psi.shape), oracle.wilson(L, links, psi, KAPPA, dagger=bool(dagger))) <= gate
    g.close()


def clover_storage_model(A):
    """The clover term as FP16/BF16 launches read it: two Hermitian 6x6 blocks
    per site (spins 0-1 and 2-3, all colours), the 6 real diagonal entries and
    the 15 complex entries above the diagonal each rounded once from FP64 to
    the nearest FP16 value, the lower triangle their conjugates, nothing outside
    the blocks."""
    Aq = np.zeros_like(A)
    for b in range(2):
        blk = A[:, 6 * b:6 * b + 6, 6 * b:6 * b + 6]
        re = blk.real.astype(np.float16).astype(np.float64)
        im = blk.imag.astype(np.float16).astype(np.float64)
        q = re + 1j * im
        iu = np.triu_indices(6, 1)
        full = np.zeros_like(q)
        full[:, iu[0], iu[1]] = q[:, iu[0], iu[1]]
        full[:, iu[1], iu[0]] = np.conj(q[:, iu[0], iu[1]])
        d = np.arange(6)
        full[:, d, d] = re[:, d, d]
        Aq[:, 6 * b:6 * b + 6, 6 * b:6 * b + 6] = full
    return Aq


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dagger", [0, 1])
def test_clover_dslash_half_precision(links, prec, dagger):
    """FP16/BF16 storage reads the FP16 copy of the clover term.  Compared with
    the oracle's operator on the storage-rounded inputs (spinors with their site
    norm, links rebuilt from two rounded rows, the clover term's packed entries
    rounded to FP16): D psi = A psi - kappa H psi, with the oracle's A and H.
    What remains is the output's rounding to storage, at most half a unit of a
    value in [0.5, 1] times the site maximum (2^-12 FP16, 2^-9 BF16), plus the
    FP32 arithmetic: per site, on the 24 reals, 1.01 x that + 1e-5 of the
    field's mean site maximum."""
    w = need_gpu()
    psi = li.gaussian_spinor(L, 2305, nrhs=2)
    V = li.volume(L)
    pq = quantize_spinor(psi, prec)
    Uq = quantize_links(links, prec, 12)
    Aq = clover_storage_model(oracle.clover(L, links, KAPPA, CSW))
    Apsi = np.einsum("vij,rvj->rvi", Aq, pq.reshape(2, V, 12)).reshape(psi.shape)
    ref = Apsi - KAPPA * oracle.hop(L, Uq, pq, dagger=bool(dagger))
    g = w.Gauge(L, to_dev(links))
    out = to_dev(np.zeros_like(psi))
    w.wilson_clover_dslash(g, to_dev(psi), out, 2, KAPPA, CSW, dagger, prec, 12)
    got = from_dev(out, psi.shape)
    e = half_storage_excess(got, ref, prec)
    assert e <= 1e-5, (prec, dagger, e)
    g.close()


@pytest.mark.parametrize("method", ["cg", "bicgstab"])
@pytest.mark.parametrize("sloppy,recon", [("f64", 18), ("f32", 12), ("f16", 12), ("bf16", 12)])
def test_clover_solve_matches_oracle(links, method, sloppy, recon):
    w = need_gpu()
    tol = 1e-10
    eta = li.gaussian_spinor(L, 2302, nrhs=2)
    g = w.Gauge(L, to_dev(links))
    x = to_dev(np.zeros_like(eta))
    solve = w.wilson_clover_cg if method == "cg" else w.wilson_clover_bicgstab
    st, info = solve(g, to_dev(eta), x, 2, KAPPA, CSW, tol, 3000, sloppy, recon, 0.1)
    got = from_dev(x, eta.shape)
    ref, conv, iters, res = oracle.cg_eo_clover(L, links, eta, KAPPA, CSW, tol=1e-12)
    assert conv
    for r in range(2):
        assert info[r]["converged"] == 1 and info[r]["true_resid"] <= tol, info[r]
        # the oracle's whole-lattice clover operator confirms the residual
        resid = rel(oracle.wilson_clover(L, links, got[r], KAPPA, CSW), eta[r])
        assert resid <= 1.5 * tol, (r, resid)
        assert rel(got[r], ref[r]) <= 1e-8, (r, rel(got[r], ref[r]))
    g.close()


def test_clover_fullsize_f16_cg():
    """16^3 x 32 (65536 sites per parity), FP16 sloppy with FP32 clover term:
    the oracle's operator confirms the true residual."""
    w = need_gpu()
    Lb = (16, 16, 16, 32)
    U = li.near_identity_links(Lb, 0.3, 1302)
    eta = li.gaussian_spinor(Lb, 2303)
    g = w.Gauge(Lb, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.wilson_clover_cg(g, to_dev(eta), x, 1, 0.124, 1.0, 1e-10, 5000, "f16", 12, 0.1)
    got = from_dev(x, eta.shape)
    assert info[0]["converged"] == 1 and info[0]["true_resid"] <= 1e-10, info[0]
    assert rel(oracle.wilson_clover(Lb, U, got[0], 0.124, 1.0), eta[0]) <= 1.5e-10
    g.close()


def test_clover_validation(links):
    w = need_gpu()
    eta = li.gaussian_spinor(L, 2304)
    g = w.Gauge(L, to_dev(links))
    x = to_dev(np.zeros_like(eta))
    with pytest.raises(w.WilsonError) as e:
        w.wilson_clover_cg(g, to_dev(eta), x, 1, KAPPA, -1.0, 1e-10, 100, "f32", 12, 0.1)
    assert e.value.status == w.WL_ERR_ARG
    with pytest.raises(w.WilsonError) as e:
        w.wilson_clover_dslash(g, to_dev(eta), x, 1, KAPPA, CSW, 0, "f16", 18)
    assert e.value.status == w.WL_ERR_PREC
    g.close()


@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f32", 12), ("f16", 12), ("bf16", 12)])
def test_clover_variants_agree_bitwise(links, prec, recon, monkeypatch):
    """The clover epilogue writes out its fused multiply-adds, so every launch
    variant that runs it (fence 2 with non-temporal or cached links; for half
    precision also fence 4) gives the same operator bit for bit."""
    w = need_gpu()
    psi = li.gaussian_spinor(L, 2302, nrhs=2)
    cfgs = ["0:256", "0:64", "3:512", "3:1024:16"] + (["4:256", "5:128"] if prec in ("f16", "bf16") else [])
    for dagger in (0, 1):
        ref = None
        for c in cfgs:
            monkeypatch.setenv("WL_TUNE_FORCE", c)
            g = w.Gauge(L, to_dev(links))
            out = to_dev(np.zeros_like(psi))
            w.wilson_clover_dslash(g, to_dev(psi), out, 2, KAPPA, CSW, dagger, prec, recon)
            got = from_dev(out, psi.shape)
            g.close()
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), (prec, recon, dagger, c)
