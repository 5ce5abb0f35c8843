"""GPU parity of the D-slash (single-parity hop and whole-lattice D) against the
FP64 oracle, through the C ABI, for every storage precision and compression.

Gates (relative to the oracle on the same, storage-rounded inputs):
  FP64: relative L2 error <= 1e-13
  FP32 (recon 18 or 12): <= 1e-6
  FP16 / BF16 (recon 12, per-site norm): compared with the oracle on the
  inputs rounded to storage by a host model; the extra error is the rounding
  of the output to storage (at most half a unit in the last place of the
  site-normalised value: 2^-11 for FP16, 2^-8 for BF16, of the site maximum)
  plus rare one-unit differences of the input rounding where the host model's
  FP32 value sits on a rounding boundary, plus 1e-5 for the FP32 arithmetic:
  gate 2 x 2^-11 (FP16) / 2 x 2^-8 (BF16) + 1e-5.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import from_dev, need_gpu, quantize_links, quantize_spinor, rel, site_max_err, to_dev

pytestmark = pytest.mark.gpu

GATE = {"f64": 1e-13, "f32": 1e-6}
QGATE = {"f16": 2.0 * 2.0 ** -11 + 1e-5, "bf16": 2.0 * 2.0 ** -8 + 1e-5}
CASES = [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 12), ("bf16", 12)]


def run_dslash(w, L, U, psi, kappa, parity, dagger, prec, recon, apbc=True):
    g = w.Gauge(L, to_dev(U), antiperiodic_t=apbc)
    din = to_dev(psi)
    dout = to_dev(np.full_like(psi, np.nan))  # every output element must be written
    w.wilson_dslash(g, din, dout, psi.shape[0], kappa, parity, dagger, prec, recon)
    out = from_dev(dout, psi.shape)
    g.close()
    return out


def expected(L, U, psi, kappa, parity, dagger, prec, recon, apbc=True):
    Uq = quantize_links(U, prec, recon)
    pq = quantize_spinor(psi, prec) if prec in ("f16", "bf16") else psi
    if parity >= 0:
        return oracle.hop(L, Uq, pq, out_parity=parity, dagger=dagger, antiperiodic_t=apbc)
    return oracle.wilson(L, Uq, pq, kappa, dagger=dagger, antiperiodic_t=apbc)


def check(prec, got, ref):
    assert np.all(np.isfinite(got))
    if prec in GATE:
        e = rel(got, ref)
        assert e <= GATE[prec], "%s relative error %g" % (prec, e)
    else:
        e = site_max_err(got, ref)
        assert e <= QGATE[prec], "%s site error %g" % (prec, e)
    return e


@pytest.mark.parametrize("prec,recon", CASES)
@pytest.mark.parametrize("parity", [0, 1, -1])
def test_dslash_parity_small(prec, recon, parity):
    w = need_gpu()
    L = (4, 6, 2, 8)  # non-cubic: catches index-order mistakes
    U = li.haar_links(L, 11)
    psi = li.gaussian_spinor(L, 12, nrhs=2)
    for dagger in (0, 1):
        got = run_dslash(w, L, U, psi, 0.13, parity, dagger, prec, recon)
        check(prec, got, expected(L, U, psi, 0.13, parity, dagger, prec, recon))


@pytest.mark.parametrize("L,apbc", [((2, 2, 2, 2), True), ((6, 4, 2, 10), False), ((10, 2, 6, 4), True)])
def test_dslash_ragged_and_tiny(L, apbc):
    """Sites per parity not a multiple of any block size (ragged tail), L = 2 wraps."""
    w = need_gpu()
    U = li.haar_links(L, 21)
    psi = li.gaussian_spinor(L, 22, nrhs=3)
    for prec, recon in [("f64", 18), ("f32", 12), ("f16", 12)]:
        for parity in (0, 1):
            got = run_dslash(w, L, U, psi, 0.1, parity, 0, prec, recon, apbc)
            check(prec, got, expected(L, U, psi, 0.1, parity, 0, prec, recon, apbc))


def test_dslash_point_source_half_precision():
    """Zero sites of a point source must store zero norms, not NaN."""
    w = need_gpu()
    L = (4, 4, 4, 4)
    U = li.near_identity_links(L, 0.3, 31)
    psi = li.point_sources(L)[:4]
    for prec in ("f16", "bf16"):
        got = run_dslash(w, L, U, psi, 0.12, -1, 0, prec, 12)
        check(prec, got, expected(L, U, psi, 0.12, -1, 0, prec, 12))


def test_dslash_full_size_24c48():
    """The benchmark lattice (24^3 x 48, eps = 0.3 links) in FP32 recon-12 and FP64."""
    w = need_gpu()
    L = (24, 24, 24, 48)
    U = li.near_identity_links(L, 0.3, 1002)
    psi = li.gaussian_spinor(L, 2002)
    for prec, recon, parity in [("f32", 12, 0), ("f64", 18, 1), ("f16", 12, 0)]:
        got = run_dslash(w, L, U, psi, 0.1245, parity, 0, prec, recon)
        check(prec, got, expected(L, U, psi, 0.1245, parity, 0, prec, recon))


def test_dslash_rejects_host_pointers_and_overlap():
    w = need_gpu()
    import torch

    L = (4, 4, 4, 4)
    U = li.haar_links(L, 1)
    g = w.Gauge(L, to_dev(U))
    psi = li.gaussian_spinor(L, 2)
    host = torch.from_numpy(psi.view(np.float64))
    dev = to_dev(psi)
    with pytest.raises(w.WilsonError) as e:
        w.wilson_dslash(g, host, dev, 1, 0.1, 0)
    assert e.value.status == w.WL_ERR_ARG
    with pytest.raises(w.WilsonError) as e:
        w.wilson_dslash(g, dev, dev, 1, 0.1, 0)
    assert e.value.status == w.WL_ERR_ARG
    with pytest.raises(w.WilsonError) as e:
        w.wilson_dslash(g, dev, to_dev(psi), 1, 0.1, 0, 0, "f16", 18)
    assert e.value.status == w.WL_ERR_PREC
    g.close()
