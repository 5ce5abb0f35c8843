"""GPU parity of the D-slash (single-parity hop and whole-lattice D) against the
FP64 oracle, through the C ABI, for every storage precision and compression.

Gates (against the oracle applied to the same storage-rounded inputs, whose
host model is pinned bit for bit by test_pack_quantize_bit_exact):
  FP64: relative L2 error <= 1e-13 and per-site error <= 1e-12
  FP32 (recon 18 or 12): relative L2 error <= 1e-6 and per-site error <= 1e-5
  FP16 / BF16 (recon 12, per-site norm): the output is rounded to nearest even
  after division by its site maximum m_s, which moves each real by at most half
  a unit in the last place of a value in [0.5, 1]: 2^-12 m_s for FP16 (11
  significant bits), 2^-9 m_s for BF16 (8).  Gate per site, on the 24 reals:
  max |gpu - oracle| <= 1.01 x that half unit x m_s + 1e-5 M for the FP32
  arithmetic, M the field's mean site maximum (the arithmetic error scales with
  the inputs, not with a site's own output).  An output conversion that
  truncates instead of rounding moves a value by up to a whole unit and fails.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import (from_dev, half_storage_excess, need_gpu, quantize_links, quantize_spinor, rel,
                            site_max_err_real, to_dev)

pytestmark = pytest.mark.gpu

GATE = {"f64": 1e-13, "f32": 1e-6}
SITE_GATE = {"f64": 1e-12, "f32": 1e-5}
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
        es = site_max_err_real(got, ref)
        assert es <= SITE_GATE[prec], "%s site error %g" % (prec, es)
    else:
        e = half_storage_excess(got, ref, prec)
        assert e <= 1e-5, "%s: site error exceeds the rounding bound by %g of the field scale" % (prec, e)
    return e


def _crafted_sites(L, prec):
    """Fields whose sites exercise the storage rounding: in the first, every
    site holds 1.0 and 23 values exactly halfway between two neighbouring
    half-precision numbers in [0.5, 1) (site maximum 1, so the stored value is
    the input itself and round-to-nearest-even decides each tie); in the
    second, values a factor up to 2^+-20 apart within a site, and zero sites."""
    V = li.volume(L)
    rng = np.random.default_rng(5)
    psi = li.gaussian_spinor(L, 6, nrhs=2)
    re = psi.view(np.float64).reshape(2, V, 24)
    bits = 11 if prec == "f16" else 8  # significant bits: spacing 2^-bits in [0.5, 1)
    k = rng.integers(2 ** (bits - 1), size=(V, 23))
    sgn = rng.choice([-1.0, 1.0], size=(V, 23))
    re[0, :, 0] = 1.0
    re[0, :, 1:] = sgn * (0.5 + (k + 0.5) * 2.0 ** -bits)
    re[1, ::3] *= 2.0 ** rng.integers(-20, 21, size=(len(range(0, V, 3)), 24))
    re[1, 1::7] = 0.0
    return psi


def test_pack_quantize_bit_exact():
    """wilson_dslash with parity -1 and kappa 0 returns the input after it has
    been packed, read by the epilogue (which adds the zero hopping term),
    stored and unpacked: FP64 unchanged, FP32 rounded once, FP16/BF16 quantised
    twice (v / max|v| over the site's 24 reals, rounded to nearest even, times
    the FP32 norm; see quantize_spinor for the exact order).  The result must
    equal the host model of that rounding order bit for bit, including exact
    ties and values in FP16's subnormal range and below it."""
    w = need_gpu()
    L = (4, 6, 2, 8)
    for prec, recon in CASES:
        for psi in (li.gaussian_spinor(L, 12, nrhs=2), li.point_sources(L)[:2],
                    _crafted_sites(L, prec if prec in ("f16", "bf16") else "f16")):
            got = run_dslash(w, L, li.haar_links(L, 11), psi, 0.0, -1, 0, prec, recon)
            # (the epilogue adds the zero hopping term, which turns a -0 into +0)
            if prec == "f64":
                want = psi + 0.0
            elif prec == "f32":
                want = psi.astype(np.complex64).astype(np.complex128) + 0.0
            else:
                want = quantize_spinor(quantize_spinor(psi, prec) + 0.0, prec)
            gb = np.ascontiguousarray(got).view(np.uint64)
            wb = np.ascontiguousarray(want).view(np.uint64)
            nbad = int(np.count_nonzero(gb != wb))
            assert nbad == 0, "%s: %d of %d reals differ from the storage model" % (prec, nbad, gb.size)


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
