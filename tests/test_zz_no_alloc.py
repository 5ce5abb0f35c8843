"""wilson_dslash_noalloc (the D-slash entry point that allocates nothing)
against wilson_dslash, through the C ABI: two calls in a row, the second on a
smaller lattice with fewer right-hand sides, for every storage precision and
for the single-parity hop and the whole-lattice operator.

Both entry points run the same kernels, possibly in different launch variants,
so they agree to the D-slash gates: FP64 relative L2 1e-13, FP32 1e-6; FP16 /
BF16 per site, two outputs each rounded to storage with at most half a unit of
a value in [0.5, 1] times the site maximum, plus the FP32 arithmetic, differ by
at most one such unit plus twice the arithmetic allowance.  Each output is also
checked against the oracle on the storage-rounded inputs."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import from_dev, half_storage_excess, need_gpu, quantize_links, quantize_spinor, rel, to_dev

pytestmark = pytest.mark.gpu

CASES = [("f64", 18), ("f64", 12), ("f32", 12), ("f32", 18), ("f16", 12), ("bf16", 12)]


def both(w, L, U, psi, kappa, parity, dagger, prec, recon):
    g = w.Gauge(L, to_dev(U))
    din = to_dev(psi)
    a = to_dev(np.full_like(psi, np.nan))
    b = to_dev(np.full_like(psi, np.nan))
    w.wilson_dslash(g, din, a, psi.shape[0], kappa, parity, dagger, prec, recon)
    w.wilson_dslash_noalloc(g, din, b, psi.shape[0], kappa, parity, dagger, prec, recon)
    ra, rb = from_dev(a, psi.shape), from_dev(b, psi.shape)
    g.close()
    return ra, rb


def expected(L, U, psi, kappa, parity, dagger, prec, recon):
    Uq = quantize_links(U, prec, recon)
    pq = quantize_spinor(psi, prec) if prec in ("f16", "bf16") else psi
    if parity >= 0:
        return oracle.hop(L, Uq, pq, out_parity=parity, dagger=dagger)
    return oracle.wilson(L, Uq, pq, kappa, dagger=dagger)


@pytest.mark.parametrize("prec,recon", CASES)
def test_noalloc_matches_dslash_twice(prec, recon):
    w = need_gpu()
    runs = [((8, 8, 8, 8), 2, 0, 0), ((4, 6, 2, 8), 1, -1, 1)]  # second call: smaller lattice, fewer rhs
    for n, (L, nrhs, parity, dagger) in enumerate(runs):
        U = li.near_identity_links(L, 0.3, 4100 + n)
        psi = li.gaussian_spinor(L, 4200 + n, nrhs=nrhs)
        a, b = both(w, L, U, psi, 0.1245, parity, dagger, prec, recon)
        assert np.all(np.isfinite(b))
        ref = expected(L, U, psi, 0.1245, parity, dagger, prec, recon)
        if prec in ("f64", "f32"):
            gate = 1e-13 if prec == "f64" else 1e-6
            assert rel(b, a) <= gate, (L, prec, rel(b, a))
            assert rel(b, ref) <= gate, (L, prec, rel(b, ref))
        else:
            e = half_storage_excess(b, a, prec, units=2.0, arith=2e-5)
            assert e <= 2e-5, (L, prec, e)
            e = half_storage_excess(b, ref, prec)
            assert e <= 1e-5, (L, prec, e)


def test_noalloc_rejects_what_does_not_fit():
    """A lattice whose packed links and fields exceed the fixed scratch array is
    refused before any device work; wilson_dslash serves it."""
    w = need_gpu()
    L = (24, 24, 24, 24)  # FP64 recon-18 links alone: 8 x 165,888 x 144 B = 191 MB > 128 MiB
    U = li.unit_links(L)
    psi = li.gaussian_spinor(L, 7)
    g = w.Gauge(L, to_dev(U))
    x = to_dev(psi)
    y = to_dev(np.zeros_like(psi))
    with pytest.raises(w.WilsonError) as e:
        w.wilson_dslash_noalloc(g, x, y, 1, 0.12, 0, 0, "f64", 18)
    assert e.value.status == w.WL_ERR_ARG
    assert np.abs(from_dev(y, psi.shape)).max() == 0.0
    # the same lattice in FP16 fits: links 8 x 165,888 x 24 B, two fields of 52 B per site
    w.wilson_dslash_noalloc(g, x, y, 1, 0.12, 0, 0, "f16", 12)
    ref = oracle.hop(L, quantize_links(U, "f16", 12), quantize_spinor(psi, "f16"), out_parity=0)
    assert half_storage_excess(from_dev(y, psi.shape), ref, "f16") <= 1e-5
    g.close()
