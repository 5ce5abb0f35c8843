"""The oracle's Chebyshev sign function at the full size of the sign-function
workload: 16^3 x 32, eps = 0.2 links (seed 1005), rho = 1.5, degree 200, the
spectrum of H_W^2 divided by 42.25 (a bound on lambda_max(H_W^2) for any SU(3)
field), one Gaussian right-hand side (seed 2005).

eps(H_W)^2 = 1 holds for the exact sign function.  The degree-200 interpolant
of x^-1/2 on the window [lo, 1] reproduces it to its scalar error
max |x p(x)^2 - 1| (1.8e-10 on [0.003, 1]) only where the window covers the
spectrum of H_W^2 / 42.25, whose lower end on this ensemble lies near 0.0067:
  * window [0.003, 1] (the reading the tests gate on): the FP64 residual
    |eps(eps(v)) - v| / |v| is <= 1e-8;
  * the literal window [0.01, 1] leaves the lowest modes outside, where the
    polynomial is not an approximation of x^-1/2, and the residual exceeds
    1e-8 (its value is printed and recorded in the design notes).
Each case costs the oracle 806 whole-lattice H_W applications.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle

pytestmark = pytest.mark.slow

L = (16, 16, 16, 32)
RHO, DEG, SCALE = 1.5, 200, 42.25


@pytest.fixture(scope="module")
def inputs():
    return li.near_identity_links(L, 0.2, 1005), li.gaussian_spinor(L, 2005)[0]


def eps2_residual(U, v, lo):
    e1 = oracle.sign_cheb(L, U, v, RHO, DEG, lo, 1.0, SCALE)
    e2 = oracle.sign_cheb(L, U, e1, RHO, DEG, lo, 1.0, SCALE)
    return float(np.linalg.norm(e2 - v) / np.linalg.norm(v)), float(np.linalg.norm(e1) / np.linalg.norm(v))


def test_eps_squared_gate_window(inputs):
    U, v = inputs
    r, n = eps2_residual(U, v, 0.003)
    print("\n[sign 16^3x32] window [0.003, 1]: |eps^2 v - v| / |v| = %.3e, |eps v| / |v| = %.12f" % (r, n))
    assert r <= 1e-8
    assert abs(n - 1.0) <= 1e-8


def test_eps_squared_literal_window(inputs):
    U, v = inputs
    r, n = eps2_residual(U, v, 0.01)
    print("\n[sign 16^3x32] window [0.01, 1]: |eps^2 v - v| / |v| = %.3e, |eps v| / |v| = %.12f" % (r, n))
    assert 1e-8 < r < 1e-2
