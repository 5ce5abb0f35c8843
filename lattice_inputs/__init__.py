"""Seeded synthetic inputs for the Wilson-Dirac inverter path.

This module only draws random numbers and shapes them into gauge-link and
spinor fields in the canonical layout.  It holds none of the operator, solver
or polynomial arithmetic; both the CPU oracle (in the tests) and the GPU
library consume exactly the arrays built here.

Canonical layout (complex128, (re, im) interleaved in memory):
  lattice  L = (Lx, Ly, Lz, Lt), all even; site s = x + Lx*(y + Ly*(z + Lz*t))
  links    U[s][mu][a][b]       3x3 row-major, mu = 0..3 = x, y, z, t;
                                U_mu(x) transports the field at x+mu back to x
  spinors  psi[r][s][spin][col] r = right-hand-side index (slowest)

Random draws use numpy's PCG64 (``default_rng(seed)``).  Complex Gaussians
have real and imaginary parts drawn independently from N(0, 1/2), so that
E|z|^2 = 1.  Draw order is site-lexicographic, then mu, then row-major matrix
entries, then (re, im) -- i.e. the C order of the array shapes used below.

The paper measures on real gauge configurations that are not available here;
these fields stand in for them with the same shapes and a comparable
plaquette (Table 2 gives no lattice; the overlap and multigrid runs of the
performance section used 24^3x64 and 96^3x192 ensembles).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "volume",
    "haar_links",
    "near_identity_links",
    "gaussian_spinor",
    "point_sources",
    "haar_su3_matrices",
    "unit_links",
]


def volume(L) -> int:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return Lx * Ly * Lz * Lt


def _complex_gauss(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian array, re and im ~ N(0, 1/2), drawn (re, im) innermost."""
    z = rng.standard_normal(tuple(shape) + (2,)) * math.sqrt(0.5)
    return z[..., 0] + 1j * z[..., 1]


def haar_su3_matrices(A: np.ndarray) -> np.ndarray:
    """Turn complex Gaussian 3x3 matrices into Haar-random SU(3) matrices.

    Rows 0 and 1 are Gram-Schmidt orthonormalised; row 2 is conj(row0 x row1),
    which makes the matrix special unitary.  The first two rows of a Haar U(3)
    matrix are distributed like those of a Haar SU(3) matrix, so the result is
    exactly Haar on SU(3), and its third row is what a 12-real compression
    rebuilds.
    """
    A = np.asarray(A, dtype=np.complex128)
    r0 = A[..., 0, :]
    r0 = r0 / np.sqrt(np.sum(np.abs(r0) ** 2, axis=-1, keepdims=True))
    r1 = A[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.sqrt(np.sum(np.abs(r1) ** 2, axis=-1, keepdims=True))
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def haar_links(L, seed: int) -> np.ndarray:
    """Haar-random SU(3) links, shape (V, 4, 3, 3), complex128."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    A = _complex_gauss(rng, (V, 4, 3, 3))
    return np.ascontiguousarray(haar_su3_matrices(A))


def near_identity_links(L, eps: float, seed: int) -> np.ndarray:
    """Smooth random links U = exp(i*eps*H), H random traceless Hermitian.

    H = (A + A^dagger)/sqrt(2) with A complex Gaussian, then the trace is
    removed; this is GUE-normalised (E|H_ij|^2 = 1).  The exponential is
    taken through the eigen-decomposition H = V diag(w) V^dagger.
    eps = 0.3 gives a plaquette near 0.61, eps = 0.2 near 0.81.
    """
    import torch  # batched CPU eigh is several times faster than numpy's

    V = volume(L)
    rng = np.random.default_rng(seed)
    A = _complex_gauss(rng, (V, 4, 3, 3))
    H = (A + np.conj(np.swapaxes(A, -1, -2))) / math.sqrt(2.0)
    del A
    tr = np.trace(H, axis1=-2, axis2=-1) / 3.0
    for i in range(3):
        H[..., i, i] -= tr
    w, vec = torch.linalg.eigh(torch.from_numpy(H.reshape(-1, 3, 3)))
    del H
    ph = torch.exp(1j * eps * w.to(torch.complex128))
    U = (vec * ph[..., None, :]) @ vec.conj().transpose(-1, -2)
    return np.ascontiguousarray(U.numpy().reshape(V, 4, 3, 3))


def unit_links(L) -> np.ndarray:
    """The free field U = 1 on every link."""
    V = volume(L)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_spinor(L, seed: int, nrhs: int = 1) -> np.ndarray:
    """Complex Gaussian spinor fields, shape (nrhs, V, 4, 3)."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_complex_gauss(rng, (nrhs, V, 4, 3)))


def point_sources(L, site: int = 0) -> np.ndarray:
    """The 12 spin-colour point sources at one site, shape (12, V, 4, 3).

    Right-hand side r = 3*spin + colour is the unit vector delta_{x,site}
    delta_{s,spin} delta_{c,colour}.
    """
    V = volume(L)
    eta = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            eta[3 * s + c, site, s, c] = 1.0
    return eta
