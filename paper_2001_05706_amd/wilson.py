"""Python binding of libwilson.so: argument marshalling only.

Every function has the name and argument order of the C entry point it wraps
(include/wilson.h).  Field arguments are torch tensors on the GPU holding the
canonical layout (complex128 or float64 views of the same memory); their data
pointers and the current HIP stream are passed through unchanged, and every
step of the computation runs in the HIP library.  There is no fallback: if the
library is missing or does not load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwilson.so")

WL_OK, WL_ERR_ARG, WL_ERR_GEOM, WL_ERR_PREC, WL_ERR_NOMEM, WL_ERR_HIP, WL_ERR_NOCONV, WL_ERR_NONFINITE = range(8)
WL_F64, WL_F32, WL_F16, WL_BF16 = range(4)
PREC = {"f64": WL_F64, "f32": WL_F32, "f16": WL_F16, "bf16": WL_BF16}


class WlGeom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("antiperiodic_t", ctypes.c_int32)]


class WlSolveInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("reliable_updates", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("precision_escalations", ctypes.c_int32),
        ("true_resid", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("gbytes", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class WilsonError(RuntimeError):
    def __init__(self, status, message, info=None):
        super().__init__("%s (status %d): %s" % (_status_name(status), status, message))
        self.status = status
        self.info = info


_lib = None

# (name, restype, argtypes) of every exported entry point
_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double
SIGNATURES = [
    ("wl_gauge_create", _i32, [ctypes.POINTER(WlGeom), _P, _P, ctypes.POINTER(_P)]),
    ("wl_gauge_destroy", None, [_P]),
    ("wilson_dslash", _i32, [_P, _P, _P, _i32, _d, _i32, _i32, _i32, _i32, _P]),
    ("wilson_dslash_noalloc", _i32, [_P, _P, _P, _i32, _d, _i32, _i32, _i32, _i32, _P]),
    ("wilson_cg", _i32, [_P, _P, _P, _i32, _d, _d, _i32, _i32, _i32, _d, ctypes.POINTER(WlSolveInfo), _P]),
    ("wilson_bicgstab", _i32, [_P, _P, _P, _i32, _d, _d, _i32, _i32, _i32, _d, ctypes.POINTER(WlSolveInfo), _P]),
    ("wilson_cg_multi", _i32, [_i32, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                               ctypes.POINTER(_i32), ctypes.POINTER(_d), _d, _i32, _i32, _i32, _d,
                               ctypes.POINTER(WlSolveInfo), _P]),
    ("wilson_clover_dslash", _i32, [_P, _P, _P, _i32, _d, _d, _i32, _i32, _i32, _P]),
    ("wilson_clover_cg", _i32, [_P, _P, _P, _i32, _d, _d, _d, _i32, _i32, _i32, _d, ctypes.POINTER(WlSolveInfo), _P]),
    ("wilson_clover_bicgstab", _i32, [_P, _P, _P, _i32, _d, _d, _d, _i32, _i32, _i32, _d,
                                      ctypes.POINTER(WlSolveInfo), _P]),
    ("overlap_sign_cheb", _i32, [_P, _P, _P, _i32, _d, _i32, _d, _d, _d, _i32, _i32, _i32, _P, ctypes.POINTER(_d),
                                 _P]),
    ("wl_hw_eigs", _i32, [_P, _d, _i32, _i32, _i32, _d, _i32, _d, _P, ctypes.POINTER(_d), ctypes.POINTER(_d),
                          ctypes.POINTER(_i32), _P]),
    ("overlap_dslash", _i32, [_P, _P, _P, _i32, _d, _d, _i32, _d, _d, _d, _i32, _i32, _i32, _i32, _P,
                              ctypes.POINTER(_d), _P]),
    ("overlap_cg", _i32, [_P, _P, _P, _i32, _d, _d, _i32, _d, _d, _d, _d, _i32, _i32, _i32, _d, _i32, _P,
                          ctypes.POINTER(_d), ctypes.POINTER(WlSolveInfo), _P]),
    ("wl_hw2_lmax", _i32, [_P, _d, _P, _i32, ctypes.POINTER(_d), _P]),
    ("wl_status_string", ctypes.c_char_p, [_i32]),
    ("wl_last_error", ctypes.c_char_p, []),
    ("wl_bench_dslash", _i32, [_P, _i32, _i32, _i32, _i32, _i32, _i32, ctypes.POINTER(_d), _P]),
    ("wl_bench_copy", _i32, [_i64, _i32, _i32, ctypes.POINTER(_d), _P]),
    ("wl_prof_enable", _i32, [_i32]),
    ("wl_prof_select", _i32, [_i32]),
    ("wl_prof_read", _i32, [ctypes.POINTER(_i64), ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    ("wl_hop_bytes_per_site", _d, [_i32, _i32, _i32]),
]


def lib():
    """Load libwilson.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwilson.so is not built: run python -m paper_2001_05706_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _status_name(s):
    try:
        return lib().wl_status_string(int(s)).decode()
    except Exception:  # the library may be the thing that failed to load
        return "status"


def last_error() -> str:
    return lib().wl_last_error().decode()


def _check(status, info=None):
    if status != WL_OK:
        raise WilsonError(status, last_error(), info)
    return status


def _ptr(t, what="tensor"):
    """Device pointer of a contiguous CUDA tensor (0 for None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


class Gauge:
    """Owning wrapper of a wl_gauge handle."""

    def __init__(self, L, U, antiperiodic_t=True, stream=None):
        g = WlGeom()
        for i in range(4):
            g.L[i] = int(L[i])
        g.antiperiodic_t = int(bool(antiperiodic_t))
        h = ctypes.c_void_p()
        _check(lib().wl_gauge_create(ctypes.byref(g), _ptr(U, "links"), _stream(stream), ctypes.byref(h)))
        self.handle = h.value
        self.L = tuple(int(v) for v in L)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]

    def close(self):
        if self.handle:
            lib().wl_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wl_gauge_create(L, U, antiperiodic_t=True, stream=None) -> Gauge:
    return Gauge(L, U, antiperiodic_t, stream)


def wl_gauge_destroy(g: Gauge):
    g.close()


def wilson_dslash(U: Gauge, inp, out, nrhs, kappa, parity, dagger=0, prec="f32", recon=12, stream=None):
    return _check(lib().wilson_dslash(U.handle, _ptr(inp, "in"), _ptr(out, "out"), int(nrhs), float(kappa),
                                      int(parity), int(dagger), _prec(prec), int(recon), _stream(stream)))


def wilson_dslash_noalloc(U: Gauge, inp, out, nrhs, kappa, parity, dagger=0, prec="f32", recon=12, stream=None):
    return _check(lib().wilson_dslash_noalloc(U.handle, _ptr(inp, "in"), _ptr(out, "out"), int(nrhs), float(kappa),
                                              int(parity), int(dagger), _prec(prec), int(recon), _stream(stream)))


def wilson_cg(U: Gauge, eta, x, nrhs, kappa, tol, maxiter, sloppy="f32", recon=12, delta=0.1, stream=None,
              check=True):
    infos = (WlSolveInfo * int(nrhs))()
    st = lib().wilson_cg(U.handle, _ptr(eta, "eta"), _ptr(x, "x"), int(nrhs), float(kappa), float(tol),
                         int(maxiter), _prec(sloppy), int(recon), float(delta), infos, _stream(stream))
    res = [i.as_dict() for i in infos]
    if check:
        _check(st, res)
    return st, res


def wilson_bicgstab(U: Gauge, eta, x, nrhs, kappa, tol, maxiter, sloppy="f32", recon=12, delta=0.1, stream=None,
                    check=True):
    infos = (WlSolveInfo * int(nrhs))()
    st = lib().wilson_bicgstab(U.handle, _ptr(eta, "eta"), _ptr(x, "x"), int(nrhs), float(kappa), float(tol),
                               int(maxiter), _prec(sloppy), int(recon), float(delta), infos, _stream(stream))
    res = [i.as_dict() for i in infos]
    if check:
        _check(st, res)
    return st, res


def wilson_cg_multi(Us, etas, xs, nrhs, kappas, tol, maxiter, sloppy="f32", recon=12, delta=0.1, stream=None,
                    check=True):
    n = len(Us)
    hU = (ctypes.c_void_p * n)(*[u.handle for u in Us])
    he = (ctypes.c_void_p * n)(*[_ptr(e, "eta[i]") for e in etas])
    hx = (ctypes.c_void_p * n)(*[_ptr(x, "x[i]") for x in xs])
    hn = (ctypes.c_int32 * n)(*[int(v) for v in nrhs])
    hk = (ctypes.c_double * n)(*[float(v) for v in kappas])
    infos = (WlSolveInfo * int(sum(int(v) for v in nrhs)))()
    st = lib().wilson_cg_multi(n, hU, he, hx, hn, hk, float(tol), int(maxiter), _prec(sloppy), int(recon),
                               float(delta), infos, _stream(stream))
    res = [i.as_dict() for i in infos]
    if check:
        _check(st, res)
    return st, res


def wilson_clover_dslash(U: Gauge, inp, out, nrhs, kappa, csw, dagger=0, prec="f32", recon=12, stream=None):
    return _check(lib().wilson_clover_dslash(U.handle, _ptr(inp, "in"), _ptr(out, "out"), int(nrhs), float(kappa),
                                             float(csw), int(dagger), _prec(prec), int(recon), _stream(stream)))


def _clover_solve(fn, U, eta, x, nrhs, kappa, csw, tol, maxiter, sloppy, recon, delta, stream, check):
    infos = (WlSolveInfo * int(nrhs))()
    st = fn(U.handle, _ptr(eta, "eta"), _ptr(x, "x"), int(nrhs), float(kappa), float(csw), float(tol), int(maxiter),
            _prec(sloppy), int(recon), float(delta), infos, _stream(stream))
    res = [i.as_dict() for i in infos]
    if check:
        _check(st, res)
    return st, res


def wilson_clover_cg(U: Gauge, eta, x, nrhs, kappa, csw, tol, maxiter, sloppy="f32", recon=12, delta=0.1,
                     stream=None, check=True):
    return _clover_solve(lib().wilson_clover_cg, U, eta, x, nrhs, kappa, csw, tol, maxiter, sloppy, recon, delta,
                         stream, check)


def wilson_clover_bicgstab(U: Gauge, eta, x, nrhs, kappa, csw, tol, maxiter, sloppy="f32", recon=12, delta=0.1,
                           stream=None, check=True):
    return _clover_solve(lib().wilson_clover_bicgstab, U, eta, x, nrhs, kappa, csw, tol, maxiter, sloppy, recon,
                         delta, stream, check)


def overlap_sign_cheb(U: Gauge, inp, out, nrhs, rho, degree, lo, hi, scale, prec="f32", recon=12, stream=None,
                      evecs=None, evals=None):
    nev, pe, pl = _defl(evecs, evals)
    return _check(lib().overlap_sign_cheb(U.handle, _ptr(inp, "in"), _ptr(out, "out"), int(nrhs), float(rho),
                                          int(degree), float(lo), float(hi), float(scale), _prec(prec), int(recon),
                                          nev, pe, pl, _stream(stream)))


def wl_hw_eigs(U: Gauge, rho, nev, nblock, degree, tol, maxiter, scale, evecs, stream=None, check=True):
    """nev low eigenpairs of H_W into the device array evecs; returns (status, evals, resid, iters)."""
    ev = (ctypes.c_double * int(nev))()
    rs = (ctypes.c_double * int(nev))()
    it = ctypes.c_int32()
    st = lib().wl_hw_eigs(U.handle, float(rho), int(nev), int(nblock), int(degree), float(tol), int(maxiter),
                          float(scale), _ptr(evecs, "evecs"), ev, rs, ctypes.byref(it), _stream(stream))
    if check:
        _check(st)
    return st, list(ev), list(rs), it.value


def _defl(evecs, evals):
    """(nev, device pointer, host double array) of an optional deflation space."""
    if evecs is None:
        return 0, None, None
    lam = [float(v) for v in evals]
    return len(lam), _ptr(evecs, "evecs"), (ctypes.c_double * len(lam))(*lam)


def overlap_dslash(U: Gauge, inp, out, nrhs, rho, mass, degree, lo, hi, scale, dagger=0, prec="f32", recon=12,
                   stream=None, evecs=None, evals=None):
    nev, pe, pl = _defl(evecs, evals)
    return _check(lib().overlap_dslash(U.handle, _ptr(inp, "in"), _ptr(out, "out"), int(nrhs), float(rho),
                                       float(mass), int(degree), float(lo), float(hi), float(scale), int(dagger),
                                       _prec(prec), int(recon), nev, pe, pl, _stream(stream)))


def overlap_cg(U: Gauge, eta, x, nrhs, rho, mass, degree, lo, hi, scale, tol, maxiter, sloppy="f32", recon=12,
               delta=1e-3, stream=None, check=True, evecs=None, evals=None):
    nev, pe, pl = _defl(evecs, evals)
    infos = (WlSolveInfo * int(nrhs))()
    st = lib().overlap_cg(U.handle, _ptr(eta, "eta"), _ptr(x, "x"), int(nrhs), float(rho), float(mass),
                          int(degree), float(lo), float(hi), float(scale), float(tol), int(maxiter),
                          _prec(sloppy), int(recon), float(delta), nev, pe, pl, infos, _stream(stream))
    res = [i.as_dict() for i in infos]
    if check:
        _check(st, res)
    return st, res


def wl_hw2_lmax(U: Gauge, rho, v0, iters, stream=None) -> float:
    r = ctypes.c_double()
    _check(lib().wl_hw2_lmax(U.handle, float(rho), _ptr(v0, "v0"), int(iters), ctypes.byref(r), _stream(stream)))
    return r.value


def wl_bench_dslash(U: Gauge, prec="f32", recon=12, nrhs=1, parity=0, nsets=1, reps=100, stream=None) -> float:
    r = ctypes.c_double()
    _check(lib().wl_bench_dslash(U.handle, _prec(prec), int(recon), int(nrhs), int(parity), int(nsets), int(reps),
                                 ctypes.byref(r), _stream(stream)))
    return r.value


def wl_bench_copy(nbytes, reps=20, stream=None, mode=0) -> float:
    """mode 0: non-temporal copy, 1: cached copy, 2: cached read-only."""
    r = ctypes.c_double()
    _check(lib().wl_bench_copy(int(nbytes), int(reps), int(mode), ctypes.byref(r), _stream(stream)))
    return r.value


def wl_prof_enable(on=True):
    _check(lib().wl_prof_enable(int(bool(on))))


def wl_prof_select(prec=-1):
    _check(lib().wl_prof_select(-1 if prec == -1 else _prec(prec)))


def wl_prof_read():
    """(launches, event ms, algorithmic GB, kernel ms) of the timed hop launches since the last read."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    gb = ctypes.c_double()
    kms = ctypes.c_double()
    _check(lib().wl_prof_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(gb), ctypes.byref(kms)))
    return n.value, ms.value, gb.value, kms.value


def wl_hop_bytes_per_site(prec="f32", recon=12, nrhs=1) -> float:
    return float(lib().wl_hop_bytes_per_site(_prec(prec), int(recon), int(nrhs)))
