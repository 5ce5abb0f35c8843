"""FP64 CPU oracle for the Wilson-Dirac inverter path -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.

The arithmetic lives in ``wilson_oracle.c`` (plain C99 complex, OpenMP over
independent sites); this module compiles it with gcc and wraps it for numpy
arrays in the canonical layout (see ``lattice_inputs``):
  links   (V, 4, 3, 3) complex128
  spinors (nrhs, V, 4, 3) complex128 (a (V, 4, 3) array is one field)

Definitions (the paper names the operators but prints no formula; these are
the textbook forms, each convention one of the readings in the design notes):
  * hop / dslash  -- the Wilson hopping term H and its single-parity blocks
    D_{p,1-p} (Table 1 QUDA_DIRAC_WILSON; Table 2 D-slash kernel)
  * wilson        -- D_k = 1 - kappa H
  * overlap_kernel-- H_W = g5 ((4 + m0) - H/2) with m0 = -rho, the kernel of
    the overlap operator inverted by GWU-code (Sections 1 and 3)
  * cg_eo         -- even-odd CG on the normal equations
  * sign_cheb     -- degree-d Chebyshev approximation of eps(H_W)
  * overlap       -- D_ov(m) = (rho + m/2) + (rho - m/2) g5 eps(H_W), the
    overlap operator, and overlap_cg, its CG solve on the normal equations
  * clover / wilson_clover / cg_eo_clover -- the Sheikholeslami-Wohlert
    clover term A (QUDA_DIRAC_CLOVER, Table 1), D_k = A - kappa H, and its
    even-odd CGNR on the asymmetric Schur complement
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile wilson_oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        d = ctypes.c_double
        lib.or_gamma.argtypes = [i32, P]
        lib.or_hop.argtypes = [P, i32, P, P, P, i32, i32, i32]
        lib.or_wilson.argtypes = [P, i32, P, P, P, i32, d, i32]
        lib.or_overlap_kernel.argtypes = [P, i32, P, P, P, i32, d]
        lib.or_cg_eo.argtypes = [P, i32, P, P, P, i32, d, d, i32, P, P]
        lib.or_cg_eo.restype = i32
        lib.or_cheb_coeffs.argtypes = [i32, d, d, P]
        lib.or_cheb_eval.argtypes = [i32, P, d, d, d]
        lib.or_cheb_eval.restype = d
        lib.or_sign_cheb.argtypes = [P, i32, P, P, P, i32, d, i32, d, d, d]
        lib.or_hw2_lmax.argtypes = [P, i32, P, d, P, i32]
        lib.or_hw2_lmax.restype = d
        lib.or_sign_cheb_defl.argtypes = [P, i32, P, P, P, i32, d, i32, d, d, d, i32, P, P]
        lib.or_overlap.argtypes = [P, i32, P, P, P, i32, d, d, i32, d, d, d, i32, i32, P, P]
        lib.or_overlap_cg.argtypes = [P, i32, P, P, P, i32, d, d, i32, d, d, d, d, i32, i32, P, P, P, P]
        lib.or_overlap_cg.restype = i32
        lib.or_clover.argtypes = [P, P, d, d, P]
        lib.or_wilson_clover.argtypes = [P, i32, P, P, P, i32, d, d, i32]
        lib.or_cg_eo_clover.argtypes = [P, i32, P, P, P, i32, d, d, d, i32, P, P]
        lib.or_cg_eo_clover.restype = i32
        lib.or_num_threads.restype = i32
        _lib = lib
        return lib


def _dims(L):
    a = np.ascontiguousarray(np.asarray(L, dtype=np.int32))
    if a.shape != (4,) or np.any(a < 2) or np.any(a % 2):
        raise ValueError("lattice dims must be 4 even integers >= 2, got %r" % (L,))
    return a


def _field(psi, V):
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    if a.shape == (V, 4, 3):
        a = a[None]
    if a.ndim != 4 or a.shape[1:] != (V, 4, 3):
        raise ValueError("spinor must have shape (nrhs, V, 4, 3) or (V, 4, 3)")
    return a


def _links(U, V):
    a = np.ascontiguousarray(U, dtype=np.complex128)
    if a.shape != (V, 4, 3, 3):
        raise ValueError("links must have shape (V, 4, 3, 3)")
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (OpenMP's own setter,
    reached through the library's handle; used to time the oracle on one core)."""
    fn = _load().omp_set_num_threads
    fn.argtypes = [ctypes.c_int]
    fn(int(n))


def gamma(mu: int) -> np.ndarray:
    """The oracle's gamma matrix: mu = 0..3 (x, y, z, t), 4 = gamma_5."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().or_gamma(int(mu), _p(out))
    return out


def hop(L, U, psi, out_parity: int = -1, dagger: bool = False, antiperiodic_t: bool = True):
    """H psi (or H^dagger psi) on the output sites of ``out_parity`` (-1: all).

    out_parity = p gives the single-parity hop D_{p,1-p}: only the
    opposite-parity sites of psi are read, and the other output sites are 0.
    """
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(psi, V)
    out = np.empty_like(a)
    _load().or_hop(_p(L), int(antiperiodic_t), _p(U), _p(a), _p(out), a.shape[0], int(out_parity), int(dagger))
    return out.reshape(np.shape(psi))


def wilson(L, U, psi, kappa: float, dagger: bool = False, antiperiodic_t: bool = True):
    """D_k psi = psi - kappa H psi on the whole lattice."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(psi, V)
    out = np.empty_like(a)
    _load().or_wilson(_p(L), int(antiperiodic_t), _p(U), _p(a), _p(out), a.shape[0], float(kappa), int(dagger))
    return out.reshape(np.shape(psi))


def overlap_kernel(L, U, psi, rho: float, antiperiodic_t: bool = True):
    """H_W psi = g5 ((4 - rho) psi - H psi / 2) on the whole lattice."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(psi, V)
    out = np.empty_like(a)
    _load().or_overlap_kernel(_p(L), int(antiperiodic_t), _p(U), _p(a), _p(out), a.shape[0], float(rho))
    return out.reshape(np.shape(psi))


def cg_eo(L, U, eta, kappa: float, tol: float, maxiter: int = 10000, x0=None, antiperiodic_t: bool = True):
    """Solve D_k psi = eta by even-odd CGNR.

    Returns (psi, converged, iters[nrhs], true_resid[nrhs]) where true_resid is
    |eta - D_k psi| / |eta| with the whole-lattice operator.
    """
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    e = _field(eta, V)
    x = np.zeros_like(e) if x0 is None else _field(x0, V).copy()
    nrhs = e.shape[0]
    iters = np.zeros(nrhs, dtype=np.int32)
    res = np.zeros(nrhs, dtype=np.float64)
    st = _load().or_cg_eo(_p(L), int(antiperiodic_t), _p(U), _p(e), _p(x), nrhs, float(kappa), float(tol),
                          int(maxiter), _p(iters), _p(res))
    return x.reshape(np.shape(eta)), st == 0, iters, res


def cheb_coeffs(degree: int, lo: float, hi: float) -> np.ndarray:
    c = np.zeros(degree + 1, dtype=np.float64)
    _load().or_cheb_coeffs(int(degree), float(lo), float(hi), _p(c))
    return c


def cheb_eval(c: np.ndarray, lo: float, hi: float, x: float) -> float:
    c = np.ascontiguousarray(c, dtype=np.float64)
    return float(_load().or_cheb_eval(len(c) - 1, _p(c), float(lo), float(hi), float(x)))


def sign_cheb(L, U, psi, rho: float, degree: int, lo: float, hi: float, scale: float, antiperiodic_t: bool = True):
    """eps(H_W) psi ~= scale^{-1/2} H_W p(H_W^2/scale) psi (Chebyshev, degree d)."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(psi, V)
    out = np.empty_like(a)
    _load().or_sign_cheb(_p(L), int(antiperiodic_t), _p(U), _p(a), _p(out), a.shape[0], float(rho), int(degree),
                         float(lo), float(hi), float(scale))
    return out.reshape(np.shape(psi))


def hw2_lmax(L, U, rho: float, v0, iters: int = 200, antiperiodic_t: bool = True) -> float:
    """Largest eigenvalue of H_W^2 by power iteration from v0 (one field)."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(v0, V)[0].copy()
    return float(_load().or_hw2_lmax(_p(L), int(antiperiodic_t), _p(U), float(rho), _p(a), int(iters)))


def _deflation(evecs, evals, V):
    """(nev, evecs array, evals array) for the C calls; nev = 0 without deflation."""
    if evecs is None:
        return 0, None, None
    ev = _field(evecs, V)
    lam = np.ascontiguousarray(evals, dtype=np.float64)
    if lam.shape != (ev.shape[0],):
        raise ValueError("one eigenvalue per eigenvector")
    return ev.shape[0], ev, lam


def sign_cheb_defl(L, U, psi, rho: float, degree: int, lo: float, hi: float, scale: float, evecs, evals,
                   antiperiodic_t: bool = True):
    """eps(H_W) psi with the eigenpairs (evecs, evals) of H_W treated exactly and
    the Chebyshev polynomial on their orthogonal complement."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(psi, V)
    nev, ev, lam = _deflation(evecs, evals, V)
    out = np.empty_like(a)
    _load().or_sign_cheb_defl(_p(L), int(antiperiodic_t), _p(U), _p(a), _p(out), a.shape[0], float(rho), int(degree),
                              float(lo), float(hi), float(scale), nev, _p(ev) if nev else None,
                              _p(lam) if nev else None)
    return out.reshape(np.shape(psi))


def overlap(L, U, psi, rho: float, mass: float, degree: int, lo: float, hi: float, scale: float,
            dagger: bool = False, antiperiodic_t: bool = True, evecs=None, evals=None):
    """D_ov(m) psi = (rho + m/2) psi + (rho - m/2) g5 eps(H_W) psi (dagger: eps g5);
    with (evecs, evals) the sign function is deflated by those eigenpairs of H_W."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(psi, V)
    nev, ev, lam = _deflation(evecs, evals, V)
    out = np.empty_like(a)
    _load().or_overlap(_p(L), int(antiperiodic_t), _p(U), _p(a), _p(out), a.shape[0], float(rho), float(mass),
                       int(degree), float(lo), float(hi), float(scale), int(dagger), nev, _p(ev) if nev else None,
                       _p(lam) if nev else None)
    return out.reshape(np.shape(psi))


def overlap_cg(L, U, eta, rho: float, mass: float, degree: int, lo: float, hi: float, scale: float, tol: float,
               maxiter: int = 10000, x0=None, antiperiodic_t: bool = True, evecs=None, evals=None):
    """Solve D_ov(m) psi = eta by CGNR with the Chebyshev sign function (deflated
    by (evecs, evals) when given).

    Returns (psi, converged, iters[nrhs], resid[nrhs]), resid = |eta - D_ov psi| / |eta|.
    """
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    e = _field(eta, V)
    x = np.zeros_like(e) if x0 is None else _field(x0, V).copy()
    nrhs = e.shape[0]
    nev, ev, lam = _deflation(evecs, evals, V)
    iters = np.zeros(nrhs, dtype=np.int32)
    res = np.zeros(nrhs, dtype=np.float64)
    st = _load().or_overlap_cg(_p(L), int(antiperiodic_t), _p(U), _p(e), _p(x), nrhs, float(rho), float(mass),
                               int(degree), float(lo), float(hi), float(scale), float(tol), int(maxiter), nev,
                               _p(ev) if nev else None, _p(lam) if nev else None, _p(iters), _p(res))
    return x.reshape(np.shape(eta)), st == 0, iters, res


def clover(L, U, kappa: float, csw: float) -> np.ndarray:
    """A(x) = 1 + i kappa c_sw sum_{m<n} s_mn F_mn(x) per site: shape (V, 12, 12),
    row/column index 3 * spin + colour."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    out = np.zeros((V, 12, 12), dtype=np.complex128)
    _load().or_clover(_p(L), _p(U), float(kappa), float(csw), _p(out))
    return out


def wilson_clover(L, U, psi, kappa: float, csw: float, dagger: bool = False, antiperiodic_t: bool = True):
    """D_k psi = A psi - kappa H psi (dagger: A psi - kappa H^dagger psi), whole lattice."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    a = _field(psi, V)
    out = np.empty_like(a)
    _load().or_wilson_clover(_p(L), int(antiperiodic_t), _p(U), _p(a), _p(out), a.shape[0], float(kappa),
                             float(csw), int(dagger))
    return out.reshape(np.shape(psi))


def cg_eo_clover(L, U, eta, kappa: float, csw: float, tol: float, maxiter: int = 10000, x0=None,
                 antiperiodic_t: bool = True):
    """Solve (A - kappa H) psi = eta by even-odd CGNR on A_ee - kappa^2 D_eo A_oo^-1 D_oe.

    Returns (psi, converged, iters[nrhs], true_resid[nrhs]) as cg_eo."""
    L = _dims(L)
    V = int(np.prod(L))
    U = _links(U, V)
    e = _field(eta, V)
    x = np.zeros_like(e) if x0 is None else _field(x0, V).copy()
    nrhs = e.shape[0]
    iters = np.zeros(nrhs, dtype=np.int32)
    res = np.zeros(nrhs, dtype=np.float64)
    st = _load().or_cg_eo_clover(_p(L), int(antiperiodic_t), _p(U), _p(e), _p(x), nrhs, float(kappa), float(csw),
                                 float(tol), int(maxiter), _p(iters), _p(res))
    return x.reshape(np.shape(eta)), st == 0, iters, res
