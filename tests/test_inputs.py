"""Checks of the seeded input generators (CPU only)."""
import numpy as np
import pytest

import lattice_inputs as li


def plaquette(L, U):
    """Average of Re Tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ / 3 over x and mu < nu."""
    Lx, Ly, Lz, Lt = L
    V = li.volume(L)
    s = np.arange(V)
    c = np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)

    def shift(mu):
        cn = c.copy()
        cn[:, mu] = (cn[:, mu] + 1) % L[mu]
        return cn[:, 0] + Lx * (cn[:, 1] + Ly * (cn[:, 2] + Lz * cn[:, 3]))

    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = U[:, mu] @ U[shift(mu), nu]
            b = U[shift(nu), mu] @ U[:, nu]
            P = a @ np.conj(np.swapaxes(b, -1, -2))
            tot += np.real(np.trace(P, axis1=-2, axis2=-1)).mean() / 3.0
    return tot / 6.0


def su3_defects(U):
    M = U.reshape(-1, 3, 3)
    unit = np.abs(np.conj(np.swapaxes(M, -1, -2)) @ M - np.eye(3)).max()
    det = np.abs(np.linalg.det(M) - 1).max()
    return unit, det


def test_haar_links_are_su3_with_haar_moments():
    L = (8, 8, 8, 8)
    U = li.haar_links(L, 1001)
    unit, det = su3_defects(U)
    assert unit < 1e-14 and det < 1e-14
    M = U.reshape(-1, 3, 3)
    n = M.shape[0]
    # E|U_ij|^2 = 1/3, E Tr U = 0, E|Tr U|^2 = 1 (statistical, ~5 sigma)
    assert abs((np.abs(M) ** 2).mean() - 1 / 3) < 5 * 0.25 / np.sqrt(9 * n)
    tr = np.trace(M, axis1=-2, axis2=-1)
    assert abs(tr.mean()) < 5 / np.sqrt(n)
    assert abs((np.abs(tr) ** 2).mean() - 1) < 5 * 1.0 / np.sqrt(n)
    # third row is what the 12-real compression rebuilds
    assert np.abs(M[:, 2] - np.conj(np.cross(M[:, 0], M[:, 1]))).max() < 1e-15


@pytest.mark.parametrize("eps,plaq", [(0.3, 0.612), (0.2, 0.806)])
def test_near_identity_links_plaquette(eps, plaq):
    L = (8, 8, 8, 8)
    U = li.near_identity_links(L, eps, 1002)
    unit, det = su3_defects(U)
    assert unit < 1e-13 and det < 1e-13
    assert abs(plaquette(L, U) - plaq) < 0.005


def test_generators_are_seeded_and_shaped():
    L = (4, 4, 4, 8)
    a = li.gaussian_spinor(L, 7, nrhs=3)
    b = li.gaussian_spinor(L, 7, nrhs=3)
    assert a.shape == (3, 512, 4, 3) and np.array_equal(a, b)
    assert not np.array_equal(a, li.gaussian_spinor(L, 8, nrhs=3))
    assert abs((np.abs(a) ** 2).mean() - 1.0) < 0.05
    ps = li.point_sources(L)
    assert ps.shape == (12, 512, 4, 3) and ps.sum() == 12
    for r in range(12):
        assert ps[r, 0, r // 3, r % 3] == 1
    assert np.array_equal(li.haar_links(L, 3), li.haar_links(L, 3))
