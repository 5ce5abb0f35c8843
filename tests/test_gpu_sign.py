"""GPU Chebyshev sign function of the overlap kernel and GPU power iteration,
through the C ABI, against the FP64 oracle (same polynomial, same scale)."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import from_dev, need_gpu, rel, to_dev

pytestmark = pytest.mark.gpu


def test_power_iteration_matches_oracle():
    w = need_gpu()
    L = (4, 4, 4, 8)
    U = li.near_identity_links(L, 0.2, 1005)
    v0 = li.gaussian_spinor(L, 7)
    g = w.Gauge(L, to_dev(U))
    got = w.wl_hw2_lmax(g, 1.5, to_dev(v0), 50)
    ref = oracle.hw2_lmax(L, U, 1.5, v0[0], iters=50)
    assert abs(got - ref) / ref <= 1e-12
    g.close()


@pytest.mark.parametrize("prec,recon,gate", [("f64", 18, 1e-12), ("f32", 12, 1e-5), ("f32", 18, 1e-5)])
def test_sign_matches_oracle(prec, recon, gate):
    w = need_gpu()
    L = (4, 4, 4, 8)
    U = li.near_identity_links(L, 0.2, 1005)
    psi = li.gaussian_spinor(L, 2005, nrhs=3)
    scale = 1.02 * oracle.hw2_lmax(L, U, 1.5, psi[0], iters=200)
    lo, hi, deg = 0.003, 1.0, 200
    ref = oracle.sign_cheb(L, U, psi, 1.5, deg, lo, hi, scale)
    g = w.Gauge(L, to_dev(U))
    out = to_dev(np.zeros_like(psi))
    w.overlap_sign_cheb(g, to_dev(psi), out, 3, 1.5, deg, lo, hi, scale, prec, recon)
    got = from_dev(out, psi.shape)
    assert rel(got, ref) <= gate, rel(got, ref)
    # eps^2 = 1 on the GPU result, to the precision of the arithmetic
    out2 = to_dev(np.zeros_like(psi))
    w.overlap_sign_cheb(g, to_dev(got), out2, 3, 1.5, deg, lo, hi, scale, prec, recon)
    assert rel(from_dev(out2, psi.shape), psi) <= (1e-9 if prec == "f64" else 1e-4)
    g.close()


def test_sign_automatic_scale():
    """scale <= 0: the library estimates lambda_max itself; the sign is unchanged."""
    w = need_gpu()
    L = (4, 4, 4, 4)
    U = li.near_identity_links(L, 0.2, 1006)
    psi = li.gaussian_spinor(L, 2006)
    g = w.Gauge(L, to_dev(U))
    out = to_dev(np.zeros_like(psi))
    w.overlap_sign_cheb(g, to_dev(psi), out, 1, 1.5, 200, 0.003, 1.0, -1.0, "f64", 18)
    got = from_dev(out, psi.shape)
    out2 = to_dev(np.zeros_like(psi))
    w.overlap_sign_cheb(g, to_dev(got), out2, 1, 1.5, 200, 0.003, 1.0, -1.0, "f64", 18)
    assert rel(from_dev(out2, psi.shape), psi) <= 1e-8
    g.close()


@pytest.mark.parametrize("prec,recon,gate", [("f64", 18, 1e-12), ("f32", 12, 1e-5)])
def test_sign_single_rhs_matches_oracle(prec, recon, gate):
    """One right-hand side: both output parities of every H_W application run
    in one launch.  A ragged lattice (6 x 4 x 2 x 10: 240 sites per parity)
    leaves a partial block in each half of that launch."""
    w = need_gpu()
    L = (6, 4, 2, 10)
    U = li.near_identity_links(L, 0.2, 1007)
    psi = li.gaussian_spinor(L, 2007)
    scale = 1.02 * oracle.hw2_lmax(L, U, 1.5, psi[0], iters=200)
    ref = oracle.sign_cheb(L, U, psi, 1.5, 100, 0.003, 1.0, scale)
    g = w.Gauge(L, to_dev(U))
    out = to_dev(np.zeros_like(psi))
    w.overlap_sign_cheb(g, to_dev(psi), out, 1, 1.5, 100, 0.003, 1.0, scale, prec, recon)
    got = from_dev(out, psi.shape)
    assert rel(got, ref) <= gate, rel(got, ref)
    g.close()


@pytest.mark.parametrize("nrhs", [1, 3])
def test_sign_streamed_fields_match_plain(nrhs, monkeypatch):
    """The hops' epilogue fields are read non-temporally for sets large
    against the last-level cache; forced on and forced off (WL_STREAM_FIELDS)
    the sign function gives bit-identical results (one right-hand side runs
    the two-parity launches, three the per-parity ones)."""
    w = need_gpu()
    L = (4, 4, 4, 8)
    U = li.near_identity_links(L, 0.2, 1005)
    psi = li.gaussian_spinor(L, 2006, nrhs=nrhs)
    scale = 1.02 * oracle.hw2_lmax(L, U, 1.5, psi[0], iters=200)

    def run():
        g = w.Gauge(L, to_dev(U))
        out = to_dev(np.zeros_like(psi))
        w.overlap_sign_cheb(g, to_dev(psi), out, nrhs, 1.5, 60, 0.003, 1.0, scale, "f32", 12)
        got = from_dev(out, psi.shape)
        g.close()
        return got

    monkeypatch.setenv("WL_STREAM_FIELDS", "0")
    a = run()
    monkeypatch.setenv("WL_STREAM_FIELDS", "1")
    b = run()
    assert np.array_equal(a, b)
    ref = oracle.sign_cheb(L, U, psi, 1.5, 60, 0.003, 1.0, scale)
    assert rel(b, ref) <= 1e-5, rel(b, ref)
