"""Every launch variant the autotuner may pick for the hop (direction fence,
occupancy target, non-temporal or cached links) x block size x column height
of the block order, pinned one at a time, must give the oracle's D-slash and a
converging mixed-precision solve."""
import os

import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import from_dev, need_gpu, to_dev
from tests.test_gpu_dslash import CASES, check, expected, run_dslash

pytestmark = pytest.mark.gpu


@pytest.fixture
def force(monkeypatch):
    def set_cfg(var, block, col=4):
        monkeypatch.setenv("WL_TUNE_FORCE", "%d:%d:%d" % (var, block, col))
    return set_cfg


@pytest.mark.parametrize("var,block,col", [(v, b, 4) for v in range(6) for b in (64, 512)] +
                         [(v, 1024, 16) for v in range(6)] + [(6, 256, 4), (6, 512, 16), (7, 64, 4), (7, 256, 16)] +
                         [(8, 256, 4), (8, 512, 16), (8, 768, 1), (8, 1024, 16)])
def test_every_hop_variant_matches_oracle(var, block, col, force):
    """(1024-thread blocks and variant 8 exist for FP32 and half-precision
    storage only; for FP64 the pinned configuration is not a candidate and the
    tuner's is used)"""
    w = need_gpu()
    force(var, block, col)
    L = (4, 6, 2, 8)
    U = li.haar_links(L, 41)
    psi = li.gaussian_spinor(L, 42, nrhs=3)
    for prec, recon in CASES:
        for parity, dagger in [(0, 0), (1, 1), (-1, 0), (-1, 1)]:
            got = run_dslash(w, L, U, psi, 0.13, parity, dagger, prec, recon)
            check(prec, got, expected(L, U, psi, 0.13, parity, dagger, prec, recon))


@pytest.mark.parametrize("var", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("sloppy", ["f16", "bf16"])
def test_every_hop_variant_solves(var, sloppy, force):
    w = need_gpu()
    force(var, 256)
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1002)
    eta = li.gaussian_spinor(L, 2002)
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.wilson_cg(g, to_dev(eta), x, 1, 0.1245, 1e-10, 2000, sloppy, 12, 0.1, check=False)
    psi = from_dev(x, eta.shape)
    g.close()
    r = eta - oracle.wilson(L, U, psi, 0.1245)
    tr = np.linalg.norm(r) / np.linalg.norm(eta)
    assert st == w.WL_OK and tr <= 1e-10, (var, sloppy, st, info, tr)


@pytest.mark.parametrize("var,block", [(6, 256), (6, 512), (7, 64), (7, 256), (8, 256), (8, 512), (8, 768),
                                       (8, 1024)])
@pytest.mark.parametrize("sloppy", ["f32", "f16"])
def test_rhs_block_variant_solves(var, block, sloppy, force):
    """variants 6 and 8 (the waves of a block serve consecutive right-hand
    sides; 8 with the block's links staged in LDS) and 7 (each thread serves
    two right-hand sides): 5 right-hand sides, so the last block of 4, 8, 12 or
    16, or the last pair, is partly empty; converged right-hand sides drop out
    one by one (a variant 8 block whose right-hand sides have all converged
    returns before staging)"""
    w = need_gpu()
    force(var, block)
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1003)
    eta = li.gaussian_spinor(L, 2003, nrhs=5)
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.wilson_cg(g, to_dev(eta), x, 5, 0.1245, 1e-10, 2000, sloppy, 12, 0.1, check=False)
    psi = from_dev(x, eta.shape)
    g.close()
    for r in range(5):
        tr = np.linalg.norm(eta[r] - oracle.wilson(L, U, psi[r], 0.1245)) / np.linalg.norm(eta[r])
        assert st == w.WL_OK and tr <= 1e-10, (block, sloppy, r, st, info[r], tr)


def test_untuned_fallback_solves(monkeypatch):
    """With tuning switched off the hop runs the fallback configuration (the
    one also used when a hop is first met inside a graph capture); a lattice
    no other test uses, so no tuned configuration is cached for it."""
    w = need_gpu()
    monkeypatch.setenv("WL_TUNE", "0")
    L = (6, 6, 4, 10)
    U = li.near_identity_links(L, 0.3, 1004)
    eta = li.gaussian_spinor(L, 2004, nrhs=2)
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.wilson_cg(g, to_dev(eta), x, 2, 0.1245, 1e-10, 2000, "f16", 12, 0.1, check=False)
    psi = from_dev(x, eta.shape)
    g.close()
    for r in range(2):
        tr = np.linalg.norm(eta[r] - oracle.wilson(L, U, psi[r], 0.1245)) / np.linalg.norm(eta[r])
        assert st == w.WL_OK and tr <= 1e-10, (r, st, info[r], tr)


@pytest.mark.parametrize("var,block", [(6, 256), (7, 64), (8, 256), (8, 768)])
def test_rhs_block_variant_two_systems(var, block, force):
    """Right-hand-side blocks across a set of two systems (3 and 5 right-hand
    sides, different lattices and kappas): a block's waves or pairs must not
    run into the next system's vectors, and a variant 8 block that holds all
    right-hand sides of its system reads its links non-temporally."""
    w = need_gpu()
    force(var, block)
    L1, L2 = (8, 8, 8, 8), (4, 6, 4, 8)
    U1 = li.near_identity_links(L1, 0.3, 1006)
    U2 = li.near_identity_links(L2, 0.3, 1007)
    e1 = li.gaussian_spinor(L1, 2006, nrhs=3)
    e2 = li.gaussian_spinor(L2, 2007, nrhs=5)
    g1, g2 = w.Gauge(L1, to_dev(U1)), w.Gauge(L2, to_dev(U2))
    x1, x2 = to_dev(np.zeros_like(e1)), to_dev(np.zeros_like(e2))
    st, info = w.wilson_cg_multi([g1, g2], [to_dev(e1), to_dev(e2)], [x1, x2], [3, 5], [0.1245, 0.124], 1e-10,
                                 2000, "f32", 12, 0.1)
    p1, p2 = from_dev(x1, e1.shape), from_dev(x2, e2.shape)
    g1.close()
    g2.close()
    assert st == w.WL_OK, (st, info)
    for L, U, e, p, kappa in ((L1, U1, e1, p1, 0.1245), (L2, U2, e2, p2, 0.124)):
        for r in range(e.shape[0]):
            tr = np.linalg.norm(e[r] - oracle.wilson(L, U, p[r], kappa)) / np.linalg.norm(e[r])
            assert tr <= 1e-10, (var, block, L, r, tr)


@pytest.mark.parametrize("prec,recon", [("f32", 12), ("f16", 12), ("bf16", 12), ("f32", 18), ("f64", 18)])
def test_variants_and_batching_agree_bitwise(prec, recon, monkeypatch):
    """Every launch variant runs the same per-site arithmetic in the same
    order, so they agree bit for bit: one right-hand side per thread, several
    per block (waves or pairs), links staged in LDS, every fence width and
    link-cache hint; and a 5-RHS D-slash equals five 1-RHS ones."""
    w = need_gpu()
    L = (8, 6, 4, 8)
    U = li.haar_links(L, 43)
    psi = li.gaussian_spinor(L, 44, nrhs=5)
    cfgs = ["0:256", "1:128", "2:512", "3:64", "3:1024:16", "6:256", "7:64", "8:256", "8:768"]
    if prec in ("f16", "bf16"):
        cfgs += ["4:256", "5:512"]
    for parity, dagger in [(0, 0), (1, 1), (-1, 0)]:
        ref = None
        for c in cfgs:
            monkeypatch.setenv("WL_TUNE_FORCE", c)
            got = run_dslash(w, L, U, psi, 0.13, parity, dagger, prec, recon)
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), (prec, recon, parity, dagger, c)
        monkeypatch.delenv("WL_TUNE_FORCE")
        for r in range(psi.shape[0]):
            one = run_dslash(w, L, U, psi[r:r + 1], 0.13, parity, dagger, prec, recon)
            assert np.array_equal(one[0], ref[r]), (prec, recon, parity, dagger, r)


# Pencil blocks (variants 9 and 10) need time slices of a multiple of 64 sites
# and a time extent their slice count divides: 8x8x4x8 has 128 sites per slice
# (2 chunks of 64) and 8 slices, so blocks of 2, 4 and 8 slices all tile it.
PENCIL_L = (8, 8, 4, 8)


@pytest.mark.parametrize("var,block", [(9, 128), (9, 256), (9, 512), (10, 128), (10, 256), (10, 512)])
def test_pencil_variant_matches_oracle(var, block, force):
    """(FP64 has no pencil variant: its pinned configuration is not a
    candidate and the tuner's is used)"""
    w = need_gpu()
    force(var, block)
    U = li.haar_links(PENCIL_L, 45)
    psi = li.gaussian_spinor(PENCIL_L, 46, nrhs=2)
    for prec, recon in CASES:
        for parity, dagger in [(0, 0), (1, 1), (-1, 0), (-1, 1)]:
            for apbc in (True, False):
                got = run_dslash(w, PENCIL_L, U, psi, 0.13, parity, dagger, prec, recon, apbc)
                check(prec, got, expected(PENCIL_L, U, psi, 0.13, parity, dagger, prec, recon, apbc))


@pytest.mark.parametrize("prec,recon", [("f32", 12), ("f32", 18), ("f16", 12), ("bf16", 12)])
def test_pencil_variants_agree_bitwise(prec, recon, monkeypatch):
    """Pencil blocks take the time neighbours of their inner slices from LDS and
    run the per-site arithmetic of every other variant in the same order: the
    D-slash is the same bit for bit, for every slice count and link hint."""
    w = need_gpu()
    U = li.haar_links(PENCIL_L, 47)
    psi = li.gaussian_spinor(PENCIL_L, 48, nrhs=3)
    for parity, dagger in [(0, 0), (1, 1), (-1, 0)]:
        ref = None
        for c in ["0:256", "3:256", "9:128", "9:256", "9:512", "10:128", "10:256", "10:512:16"]:
            monkeypatch.setenv("WL_TUNE_FORCE", c)
            got = run_dslash(w, PENCIL_L, U, psi, 0.13, parity, dagger, prec, recon)
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), (prec, recon, parity, dagger, c)


@pytest.mark.parametrize("var,block", [(9, 256), (10, 512)])
@pytest.mark.parametrize("sloppy", ["f32", "f16"])
def test_pencil_variant_solves(var, block, sloppy, force):
    """A mixed-precision CGNR with every sloppy hop on pencil blocks, 3
    right-hand sides (one block per vector; converged vectors drop out)."""
    w = need_gpu()
    force(var, block)
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, 0.3, 1008)
    eta = li.gaussian_spinor(L, 2008, nrhs=3)
    g = w.Gauge(L, to_dev(U))
    x = to_dev(np.zeros_like(eta))
    st, info = w.wilson_cg(g, to_dev(eta), x, 3, 0.1245, 1e-10, 2000, sloppy, 12, 0.1, check=False)
    psi = from_dev(x, eta.shape)
    g.close()
    for r in range(3):
        tr = np.linalg.norm(eta[r] - oracle.wilson(L, U, psi[r], 0.1245)) / np.linalg.norm(eta[r])
        assert st == w.WL_OK and tr <= 1e-10, (var, block, sloppy, r, st, info[r], tr)


@pytest.mark.parametrize("second", [(8, 8, 4, 8), (6, 6, 4, 10)])
def test_pencil_variant_two_systems(second, force):
    """A set of two systems: with 8x8x4x8 beside 8^4 the pinned pencil blocks
    run on both; with 6x6x4x10 (72 sites per slice) pencils cannot tile the
    second lattice, the pinned configuration is no candidate, and the tuner's
    runs instead."""
    w = need_gpu()
    force(9, 256)
    L1, L2 = (8, 8, 8, 8), second
    U1 = li.near_identity_links(L1, 0.3, 1009)
    U2 = li.near_identity_links(L2, 0.3, 1010)
    e1 = li.gaussian_spinor(L1, 2009, nrhs=2)
    e2 = li.gaussian_spinor(L2, 2010, nrhs=1)
    g1, g2 = w.Gauge(L1, to_dev(U1)), w.Gauge(L2, to_dev(U2))
    x1, x2 = to_dev(np.zeros_like(e1)), to_dev(np.zeros_like(e2))
    st, info = w.wilson_cg_multi([g1, g2], [to_dev(e1), to_dev(e2)], [x1, x2], [2, 1], [0.1245, 0.124], 1e-10,
                                 2000, "f16", 12, 0.1)
    p1, p2 = from_dev(x1, e1.shape), from_dev(x2, e2.shape)
    g1.close()
    g2.close()
    assert st == w.WL_OK, (st, info)
    for L, U, e, p, kappa in ((L1, U1, e1, p1, 0.1245), (L2, U2, e2, p2, 0.124)):
        for r in range(e.shape[0]):
            tr = np.linalg.norm(e[r] - oracle.wilson(L, U, p[r], kappa)) / np.linalg.norm(e[r])
            assert tr <= 1e-10, (second, L, r, tr)
