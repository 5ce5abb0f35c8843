"""Writes sign_16c32_samples.json: the FP64 oracle's Chebyshev sign function
eps(H_W) v (degree 200, rho = 1.5, window [0.003, 1] x 42.25) of the 12
Gaussian right-hand sides of the 16^3 x 32 workload (eps = 0.2 links, seeds
1005 / 2005), kept at sampled sites and as projections onto fixed random
fields, so that a GPU test can check every right-hand side at full size
without repeating the oracle's ~5000 whole-lattice H_W applications.

Only lattice_inputs (seeded inputs) and oracle/ are called.  Run from the
repository root:  python tests/golden/make_sign_samples.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lattice_inputs as li  # noqa: E402
import oracle  # noqa: E402

L = (16, 16, 16, 32)
RHO, DEG, LO, HI, SCALE = 1.5, 200, 0.003, 1.0, 42.25
NSITE = 32        # sampled sites per right-hand side
NPROJ = 2         # projections per right-hand side
SAMPLE_SEED = 77  # site choice and projection fields


def sample_plan():
    """Sampled sites (per RHS) and the projection fields, from a fixed seed."""
    V = li.volume(L)
    rng = np.random.default_rng(SAMPLE_SEED)
    sites = np.stack([np.sort(rng.choice(V, NSITE, replace=False)) for _ in range(12)])
    z = rng.standard_normal((NPROJ, V, 4, 3, 2)) * np.sqrt(0.5)
    w = z[..., 0] + 1j * z[..., 1]
    return sites, w


def _r(x):
    """12 significant digits: the tests compare at 1e-4 of the field's scale."""
    return float("%.12g" % x)


def main():
    U = li.near_identity_links(L, 0.2, 1005)
    v = li.gaussian_spinor(L, 2005, nrhs=12)
    ref = oracle.sign_cheb(L, U, v, RHO, DEG, LO, HI, SCALE)
    sites, w = sample_plan()
    out = {
        "what": "oracle eps(H_W) v at sampled sites and <w_j, eps(H_W) v> for 12 Gaussian rhs",
        "lattice": list(L), "links": {"eps": 0.2, "seed": 1005}, "source_seed": 2005, "nrhs": 12,
        "rho": RHO, "degree": DEG, "lo": LO, "hi": HI, "scale": SCALE, "sample_seed": SAMPLE_SEED,
        "nsite": NSITE, "nproj": NPROJ,
        "norm": [_r(np.linalg.norm(ref[k])) for k in range(12)],
        "sites": sites.tolist(),
        # values[k][i] = the 12 complex numbers of rhs k at site sites[k][i], (re, im) interleaved
        "values": [[[_r(x) for x in ref[k, s].reshape(-1).view(np.float64)] for s in sites[k]] for k in range(12)],
        # proj[k][j] = <w_j, eps(H_W) v_k> = sum conj(w_j) * ref_k, as (re, im)
        "proj": [[[_r(np.vdot(w[j], ref[k]).real), _r(np.vdot(w[j], ref[k]).imag)] for j in range(NPROJ)]
                 for k in range(12)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sign_16c32_samples.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path)


if __name__ == "__main__":
    main()
