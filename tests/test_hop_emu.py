"""CPU check of the GPU hop's per-site code (host build of the same
__host__ __device__ functions) against the FP64 oracle, before any GPU run:
packing, FP16/BF16 dequantisation, recon-12, neighbour indexing, boundary
signs, spin projection and reconstruction, for every storage precision."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests.gpu_util import quantize_links, quantize_spinor, rel

HERE = os.path.dirname(os.path.abspath(__file__))
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("emu") / "libhopemu.so")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
           "-w", os.path.join(HERE, "hop_emu.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    lib = ctypes.CDLL(out)
    lib.emu_hop.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 3 + [ctypes.c_int]
    lib.emu_hop.restype = ctypes.c_int
    lib.emu_xcd_remap.argtypes = [ctypes.c_int, ctypes.c_void_p]
    lib.emu_idiv_check.argtypes = [ctypes.c_int]
    lib.emu_idiv_check.restype = ctypes.c_long
    return lib


def run(lib, prec, recon, dag, L, U, psi, parity, apbc=True):
    Larr = np.asarray(L, dtype=np.int32)
    out = np.zeros_like(psi)
    U = np.ascontiguousarray(U)
    psi = np.ascontiguousarray(psi)
    assert lib.emu_hop(PREC[prec], recon, dag, Larr.ctypes.data, int(apbc), U.ctypes.data, psi.ctypes.data,
                       out.ctypes.data, parity) == 0
    return out


@pytest.mark.parametrize("prec,recon,gate", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 18, 1e-6),
                                             ("f32", 12, 1e-6), ("f16", 12, 3e-6), ("bf16", 12, 3e-6)])
@pytest.mark.parametrize("L,apbc", [((4, 6, 2, 8), True), ((2, 2, 2, 2), True), ((6, 4, 4, 2), False)])
def test_emulated_hop_matches_oracle(emu, prec, recon, gate, L, apbc):
    U = li.haar_links(L, 5)
    psi = li.gaussian_spinor(L, 6)[0]
    Uq = quantize_links(U, prec, recon)
    pq = quantize_spinor(psi[None], prec)[0] if prec in ("f16", "bf16") else psi
    for parity in (0, 1):
        for dag in (0, 1):
            got = run(emu, prec, recon, dag, L, U, psi, parity, apbc)
            ref = oracle.hop(L, Uq, pq, out_parity=parity, dagger=bool(dag), antiperiodic_t=apbc)
            assert rel(got, ref) <= gate, (prec, recon, parity, dag, rel(got, ref))


def test_xcd_remap_is_a_bijection(emu):
    for nb in [1, 5, 7, 8, 9, 13, 64, 1000, 1296, 5184, 12345]:
        out = np.zeros(nb, dtype=np.int32)
        emu.emu_xcd_remap(nb, out.ctypes.data)
        assert np.array_equal(np.sort(out), np.arange(nb))


def test_coordinate_division_is_exact(emu):
    """The site-coordinate code divides by the lattice extents with one FP64
    multiply-add by the reciprocal (idiv); it must equal the integer quotient
    for every extent the library accepts (up to 65536) and every checkerboard
    index below 2^26, checked at and around exact multiples."""
    assert emu.emu_idiv_check(65536) == 0
