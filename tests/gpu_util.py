"""Helpers for the GPU parity tests: device transfer of canonical fields and an
exact host model of the FP16/BF16 storage rounding, so that low-precision GPU
results can be compared with the FP64 oracle applied to the same rounded
inputs.  Nothing here computes any part of the operator."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_05706_amd import wilson

    wilson.lib()  # raises if the HIP library is missing: no silent fallback
    return wilson


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.float64)).to("cuda:0")


def from_dev(t, shape):
    return t.cpu().numpy().view(np.complex128).reshape(shape)


def bf16_round(x32):
    """float32 -> nearest-even bfloat16, returned as float32."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def round16(x32, prec):
    if prec == "f16":
        return x32.astype(np.float16).astype(np.float32)
    return bf16_round(x32)


def quantize_spinor(psi, prec):
    """What the kernels read back from a packed FP16/BF16 spinor (per-site norm),
    in the kernels' rounding order: v = FP32(input); m = max |v| over the site's
    24 reals; inv = FP32(1 / m) (correctly rounded); stored value FP16: the exact
    product v * inv rounded once to nearest even (the kernels' multiply and
    conversion are one mixed-precision fma); BF16: v * inv rounded to FP32, then
    to BF16 (the conversion is integer arithmetic on the FP32 bits); read back as
    FP32(stored * m).  A zero site stores zeros and m = 0."""
    shp = psi.shape
    v = np.ascontiguousarray(psi).view(np.float64).reshape(-1, 24).astype(np.float32)
    m = np.abs(v).max(axis=1, keepdims=True).astype(np.float32)
    safe = np.where(m > 0, m, np.float32(1))
    inv = np.where(m > 0, np.float32(1) / safe, np.float32(0)).astype(np.float32)
    if prec == "f16":
        # float32 x float32 is exact in float64; numpy rounds float64 -> float16 directly
        q = (v.astype(np.float64) * inv.astype(np.float64)).astype(np.float16).astype(np.float32)
    else:
        q = bf16_round((v * inv).astype(np.float32))
    deq = (q * m).astype(np.float32)
    return deq.astype(np.float64).view(np.complex128).reshape(shp)


def quantize_links(U, prec, recon):
    """Links as the kernels rebuild them: rows stored in prec (FP16: each real
    rounded once from FP64; BF16: to FP32, then to BF16), row 2 =
    conj(row0 x row1)."""
    Uq = np.ascontiguousarray(U).copy()
    if prec in ("f16", "bf16"):
        r = Uq.view(np.float64).reshape(U.shape[:-2] + (18,))
        r = r.astype(np.float16) if prec == "f16" else round16(r.astype(np.float32), prec)
        Uq = r.astype(np.float64).view(np.complex128).reshape(U.shape)
    elif prec == "f32":
        Uq = Uq.astype(np.complex64).astype(np.complex128)
    if recon == 12:
        Uq[..., 2, :] = np.conj(np.cross(Uq[..., 0, :], Uq[..., 1, :]))
    return Uq


def site_max_err_real(got, ref):
    """max over sites of max|got - ref| / (m_s + M) over the site's 24 reals,
    m_s the site's largest |ref| and M the field's mean site maximum: a wrong
    site scores about 1/2, the arithmetic error of a right one about the unit
    roundoff (M keeps a site whose output cancels to a small value from
    counting its inputs' rounding as its own).  Sites where the reference is
    exactly zero must be exactly zero."""
    g = np.abs(np.ascontiguousarray(got).view(np.float64).reshape(-1, 24) -
               np.ascontiguousarray(ref).view(np.float64).reshape(-1, 24)).max(axis=1)
    r = np.abs(np.ascontiguousarray(ref).view(np.float64).reshape(-1, 24)).max(axis=1)
    keep = r > 0
    assert np.all(g[~keep] == 0.0), "non-zero output where the reference site is zero"
    if not keep.any():
        return 0.0
    M = float(r[keep].mean())
    return float((g[keep] / (r[keep] + M)).max())


HALF_UNIT = {"f16": 2.0 ** -12, "bf16": 2.0 ** -9}  # half a unit of a value in [0.5, 1)


def half_storage_excess(got, ref, prec, units=1.0, arith=1e-5):
    """Check a result stored in FP16/BF16 with a per-site norm against a reference
    computed from the same storage-rounded inputs.  Rounding the output to
    storage moves each of a site's 24 reals by at most half a unit of a value in
    [0.5, 1] times the site maximum m_s (2^-12 m_s for FP16, 2^-9 m_s for BF16);
    the FP32 arithmetic adds an error on the scale of the inputs, bounded here
    by `arith` times M, the mean site maximum of the field.  Returns the largest
    excess over 1.01 x `units` x that half unit, in units of M (<= arith passes);
    sites where the reference is exactly zero must be exactly zero."""
    g = np.ascontiguousarray(got).view(np.float64).reshape(-1, 24)
    r = np.ascontiguousarray(ref).view(np.float64).reshape(-1, 24)
    err = np.abs(g - r).max(axis=1)
    m = np.abs(r).max(axis=1)
    assert np.all(err[m == 0] == 0.0), "non-zero output where the reference site is zero"
    M = float(m[m > 0].mean()) if np.any(m > 0) else 1.0
    return float(((err - 1.01 * units * HALF_UNIT[prec] * m) / M).max())


def site_max_err(got, ref):
    """max over sites of |got - ref|_inf / |ref|_inf (site-local relative error)."""
    g = np.abs(got.reshape(-1, 12) - ref.reshape(-1, 12)).max(axis=1)
    r = np.abs(ref.reshape(-1, 12)).max(axis=1)
    keep = r > 0
    return float((g[keep] / r[keep]).max()) if keep.any() else float(g.max())


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
