"""Independent dense construction of the Wilson operator for tiny lattices.

Used only to pin the oracle: the whole operator is assembled as a dense
(12V x 12V) matrix from Kronecker products of 4x4 spin and 3x3 colour blocks,
with its own site loop and gamma table, and then handed to LAPACK.

Row/column index of (site s, spin i, colour a) is 12*s + 3*i + a, so the block
coupling site x to site y is kron(spin 4x4, colour 3x3).
"""
import numpy as np

# DeGrand-Rossi basis, as stated in the conventions of the operator
GX = np.array([[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]])
GY = np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]], dtype=complex)
GZ = np.array([[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]])
GT = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]], dtype=complex)
GAMMAS = [GX, GY, GZ, GT]
G5 = np.diag([1, 1, -1, -1]).astype(complex)
ONE4 = np.eye(4, dtype=complex)


def coords(L):
    """Array of shape (V, 4) of site coordinates, x fastest."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def index(L, c):
    Lx, Ly, Lz, Lt = L
    return int(c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3])))


def hopping_matrix(L, U, antiperiodic_t=True):
    """Dense H with H psi(x) = sum_mu b(1-g_mu)U_mu(x)psi(x+mu) + b(1+g_mu)U_mu(x-mu)^+ psi(x-mu)."""
    V = int(np.prod(L))
    H = np.zeros((12 * V, 12 * V), dtype=complex)
    for x in coords(L):
        sx = index(L, x)
        for mu in range(4):
            # forward neighbour
            y = x.copy()
            y[mu] += 1
            b = 1.0
            if y[mu] == L[mu]:
                y[mu] = 0
                if mu == 3 and antiperiodic_t:
                    b = -1.0
            sy = index(L, y)
            H[12 * sx:12 * sx + 12, 12 * sy:12 * sy + 12] += b * np.kron(ONE4 - GAMMAS[mu], U[sx, mu])
            # backward neighbour: link lives on y = x - mu and is daggered
            y = x.copy()
            y[mu] -= 1
            b = 1.0
            if y[mu] < 0:
                y[mu] = L[mu] - 1
                if mu == 3 and antiperiodic_t:
                    b = -1.0
            sy = index(L, y)
            H[12 * sx:12 * sx + 12, 12 * sy:12 * sy + 12] += b * np.kron(ONE4 + GAMMAS[mu], U[sy, mu].conj().T)
    return H


def gamma5_matrix(V):
    return np.kron(np.eye(V), np.kron(G5, np.eye(3)))


def parity_mask(L):
    """Boolean mask over the 12V components: True on even sites."""
    c = coords(L)
    even = (c.sum(axis=1) % 2) == 0
    return np.repeat(even, 12)
