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
    """What the kernels read back from a packed FP16/BF16 spinor (per-site norm)."""
    shp = psi.shape
    v = np.ascontiguousarray(psi).view(np.float64).reshape(-1, 24).astype(np.float32)
    m = np.abs(v).max(axis=1, keepdims=True).astype(np.float32)
    safe = np.where(m > 0, m, np.float32(1))
    inv = np.where(m > 0, np.float32(1) / safe, np.float32(0)).astype(np.float32)
    q = round16((v * inv).astype(np.float32), prec)
    deq = (q * m).astype(np.float32)
    return deq.astype(np.float64).view(np.complex128).reshape(shp)


def quantize_links(U, prec, recon):
    """Links as the kernels rebuild them: rows stored in prec, row 2 = conj(row0 x row1)."""
    Uq = np.ascontiguousarray(U).copy()
    if prec in ("f16", "bf16"):
        r = Uq.view(np.float64).reshape(U.shape[:-2] + (18,)).astype(np.float32)
        r = round16(r, prec).astype(np.float64)
        Uq = r.view(np.complex128).reshape(U.shape)
    elif prec == "f32":
        Uq = Uq.astype(np.complex64).astype(np.complex128)
    if recon == 12:
        Uq[..., 2, :] = np.conj(np.cross(Uq[..., 0, :], Uq[..., 1, :]))
    return Uq


def site_max_err(got, ref):
    """max over sites of |got - ref|_inf / |ref|_inf (site-local relative error)."""
    g = np.abs(got.reshape(-1, 12) - ref.reshape(-1, 12)).max(axis=1)
    r = np.abs(ref.reshape(-1, 12)).max(axis=1)
    keep = r > 0
    return float((g[keep] / r[keep]).max()) if keep.any() else float(g.max())


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
