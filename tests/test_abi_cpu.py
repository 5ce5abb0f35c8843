"""The C ABI library loads and exports everything include/wilson.h declares,
and its host-side validation answers before any device work (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wilson.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(\w+)\s*\(", text, flags=re.M)) - {"if"})


@pytest.fixture(scope="module")
def w():
    from paper_2001_05706_amd import wilson

    wilson.lib()
    return wilson


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["wilson_dslash", "wilson_cg", "wilson_cg_multi", "overlap_sign_cheb", "wl_gauge_create",
              "wl_gauge_destroy", "wl_status_string", "wl_last_error"]:
        assert n in names


def test_every_declared_symbol_is_exported(w):
    lib = w.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in w.SIGNATURES}
    assert set(names) == bound


def test_status_strings_and_byte_model(w):
    lib = w.lib()
    assert lib.wl_status_string(0) == b"ok"
    assert lib.wl_status_string(6) == b"solver did not converge"
    # compulsory bytes per (site, rhs): 8 links shared by the rhs + spinor in + out
    assert w.wl_hop_bytes_per_site("f64", 18, 1) == 1536
    assert w.wl_hop_bytes_per_site("f32", 12, 1) == 576
    assert w.wl_hop_bytes_per_site("f32", 18, 1) == 768
    assert w.wl_hop_bytes_per_site("f16", 12, 1) == 296
    assert w.wl_hop_bytes_per_site("f32", 12, 12) == 224
    assert w.wl_hop_bytes_per_site("f16", 18, 1) == 0  # unsupported pair


def test_validation_before_device_work(w):
    lib = w.lib()
    h = ctypes.c_void_p()
    assert lib.wl_gauge_create(None, None, None, ctypes.byref(h)) == w.WL_ERR_ARG
    g = w.WlGeom()
    for i, v in enumerate((4, 4, 3, 4)):
        g.L[i] = v
    assert lib.wl_gauge_create(ctypes.byref(g), None, None, ctypes.byref(h)) == w.WL_ERR_GEOM
    assert "even" in w.last_error()
    assert lib.wilson_dslash(None, None, None, 1, 0.1, 0, 0, 1, 12, None) == w.WL_ERR_ARG
    info = (w.WlSolveInfo * 1)()
    assert lib.wilson_cg(None, None, None, 1, 0.1, 1e-10, 10, 1, 12, 0.1, info, None) == w.WL_ERR_ARG
    assert lib.wilson_cg_multi(0, None, None, None, None, None, 1e-10, 10, 1, 12, 0.1, info, None) == w.WL_ERR_ARG
    assert lib.overlap_sign_cheb(None, None, None, 1, 1.5, 10, 0.01, 1.0, 1.0, 1, 12, 0, None, None, None) == w.WL_ERR_ARG
    assert lib.overlap_dslash(None, None, None, 1, 1.5, 0.1, 10, 0.01, 1.0, 1.0, 0, 1, 12, 0, None, None,
                              None) == w.WL_ERR_ARG
    assert lib.overlap_cg(None, None, None, 1, 1.5, 0.1, 10, 0.01, 1.0, 1.0, 1e-8, 10, 1, 12, 1e-3, 0, None, None,
                          info, None) == w.WL_ERR_ARG
    assert lib.wilson_clover_cg(None, None, None, 1, 0.12, 1.0, 1e-10, 10, 1, 12, 0.1, info, None) == w.WL_ERR_ARG
    assert lib.wilson_clover_dslash(None, None, None, 1, 0.12, 1.0, 0, 1, 12, None) == w.WL_ERR_ARG
    ev = (ctypes.c_double * 1)()
    assert lib.wl_hw_eigs(None, 1.5, 1, 2, 8, 1e-8, 10, 1.0, None, ev, ev, None, None) == w.WL_ERR_ARG
    assert lib.wl_bench_copy(10, 1, 0, None, None) == w.WL_ERR_ARG
    sec = ctypes.c_double()
    assert lib.wl_bench_copy(1 << 20, 1, 3, ctypes.byref(sec), None) == w.WL_ERR_ARG
