"""Plant plausible mistakes in a copy of the oracle's C source and check that the
pins catch every one of them (CPU only).

Each mutant is compiled from a textual edit of wilson_oracle.c into a temporary
library, loaded through a private copy of the oracle's Python wrapper, and run
against a fast battery built from the pin tests themselves.  The committed
oracle is never modified.
"""
import importlib.util
import os
import subprocess

import numpy as np
import pytest

import lattice_inputs as li
from tests import dense_wilson as dw
from tests import test_oracle_clover as clpins
from tests import test_oracle_overlap as ovpins
from tests import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "wilson_oracle.c")

# (name, original text, mutated text)
MUTATIONS = [
    ("backward link transposed, not daggered", "conj(Umat[bb * 3 + a])", "conj(Umat[a * 3 + bb])"),
    ("backward link not conjugated", "conj(Umat[bb * 3 + a])", "Umat[bb * 3 + a]"),
    ("projector signs swapped", "const double sfwd = dagger ? +1.0 : -1.0;", "const double sfwd = dagger ? -1.0 : +1.0;"),
    ("backward link taken at x, not x-mu", "U + (yb * 4 + mu) * 9", "U + (s * 4 + mu) * 9"),
    ("antiperiodic sign dropped (forward wrap)",
     "        n[mu] = 0;\n        if (mu == 3 && g->antiperiodic_t) *bc = -1.0;", "        n[mu] = 0;\n"),
    ("antiperiodic sign dropped (backward wrap)",
     "        n[mu] = g->L[mu] - 1;\n        if (mu == 3 && g->antiperiodic_t) *bc = -1.0;",
     "        n[mu] = g->L[mu] - 1;\n"),
    ("gamma_x entry sign", "gm[2][1] = -I;", "gm[2][1] = I;"),
    ("gamma_z entry sign", "gm[1][3] = -I;", "gm[1][3] = I;"),
    ("site index stride", "(long)g->L[0] * (c[1]", "(long)g->L[1] * (c[1]"),
    ("dagger flag ignored", "or_hop(L, antiperiodic_t, U, in_, out_, nrhs, -1, dagger);",
     "or_hop(L, antiperiodic_t, U, in_, out_, nrhs, -1, 0);"),
    ("Schur operator uses kappa, not kappa^2", "vaxpby(1.0, in, -op->kappa * op->kappa, out, V * 12);",
     "vaxpby(1.0, in, -op->kappa, out, V * 12);"),
    ("even-odd source sign", "vaxpby(1.0, eta, kappa, bp, n);", "vaxpby(1.0, eta, -kappa, bp, n);"),
    ("CG beta inverted", "vaxpby(1.0, r, gam_new / gam, p, n);", "vaxpby(1.0, r, gam / gam_new, p, n);"),
    ("odd-site reconstruction sign", "x[s * 12 + k] = eta[s * 12 + k] + kappa * tmp[s * 12 + k];",
     "x[s * 12 + k] = eta[s * 12 + k] - kappa * tmp[s * 12 + k];"),
    ("overlap kernel mass sign", "vaxpby(4.0 - rho, (const cplx *)in_, -0.5, (cplx *)out_, n);",
     "vaxpby(4.0 + rho, (const cplx *)in_, -0.5, (cplx *)out_, n);"),
    ("overlap kernel missing gamma5", "    vgamma5((const cplx *)out_, (cplx *)out_, g.V * nrhs);\n}", "}"),
    ("Chebyshev nodes shifted", "double th = M_PI * (k + 0.5) / N;", "double th = M_PI * k / N;"),
    ("Clenshaw final half of c0 (scalar)", "return y * b1 - b2 + 0.5 * c[0];", "return y * b1 - b2 + c[0];"),
    ("Clenshaw final half of c0 (operator)", "w[i] = yb[i] - b2[i] + 0.5 * c[0] * v[i];", "w[i] = yb[i] - b2[i] + c[0] * v[i];"),
    ("Clenshaw recurrence sign", "b0[i] = 2.0 * yb[i] - b2[i] + c[j] * v[i];", "b0[i] = 2.0 * yb[i] + b2[i] + c[j] * v[i];"),
    ("sign function scale exponent", "1.0 / sqrt(scale), out, n);", "1.0 / scale, out, n);"),
    ("overlap mass enters both terms with one sign", "b = rho - 0.5 * mass;", "b = rho + 0.5 * mass;"),
    ("overlap missing gamma5", "            vgamma5(t, w, g.V);\n", "            memcpy(w, t, sizeof(cplx) * n);\n"),
    ("overlap adjoint equals the operator",
     "            vgamma5(v, t, g.V);\n            sign_deflated(L, antiperiodic_t, U, t, w,",
     "            vgamma5(v, t, g.V);\n            sign_deflated(L, antiperiodic_t, U, v, w,"),
    ("deflated modes keep the polynomial sign", "(evals[i] > 0 ? 1.0 : -1.0) * c[i]", "0.0 * c[i]"),
    ("deflated modes not projected out", "        vaxpby(-c[i], xi + (size_t)i * n, 1.0, w, n);\n", "\n"),
    ("overlap CG residual update sign", "            vaxpby(-alpha, q, 1.0, rt, n);\n            OV_APPLY",
     "            vaxpby(alpha, q, 1.0, rt, n);\n            OV_APPLY"),
    ("clover leaf link not daggered", "const int d1[4] = {0, 0, 1, 1};", "const int d1[4] = {0, 0, 0, 1};"),
    ("clover leaf through the wrong corner", "LK(xmm_nm, n), LK(xmm_nm, m), LK(xnm, n)",
     "LK(xmm_nm, n), LK(xnm, m), LK(xnm, n)"),
    ("clover field strength normalisation", "F[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / 8.0;",
     "F[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / 4.0;"),
    ("clover term sign", "+= I * kappa * csw * sig[m][n][i][j]", "-= I * kappa * csw * sig[m][n][i][j]"),
    ("sigma commutator reversed", "v += gm[m][i][k] * gm[n][k][j] - gm[n][i][k] * gm[m][k][j];",
     "v += gm[n][i][k] * gm[m][k][j] - gm[m][i][k] * gm[n][k][j];"),
    ("clover Schur uses A_oo, not its inverse", "        apply_site_matrix(&g, Ai, t1, t2, 1);      ",
     "        apply_site_matrix(&g, A, t1, t2, 1);       "),
    ("clover source uses A_oo, not its inverse", "apply_site_matrix(&g, Ai, eta, t1, 1);",
     "apply_site_matrix(&g, A, eta, t1, 1);"),
]


def load_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    mut = src.replace(old, new, 1)
    csrc = tmp_path / "mut.c"
    csrc.write_text(mut)
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-w", "-o", str(so), str(csrc), "-lm"],
                   check=True)
    spec = importlib.util.spec_from_file_location("oracle_mutant", os.path.join(ROOT, "oracle", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB_PATH = str(so)
    mod._lib = None
    return mod


@pytest.fixture(scope="module")
def small_cases():
    L2 = (2, 2, 2, 2)
    U2 = li.haar_links(L2, 31)
    L4 = (4, 2, 2, 4)
    U4 = li.haar_links(L4, 33)
    Lh = (2, 2, 4, 4)
    Uh = li.near_identity_links(Lh, 0.2, 35)
    kappa = 1.0 / 5.0
    V = li.volume(Lh)
    D = np.eye(12 * V) - kappa * dw.hopping_matrix(Lh, Uh)
    HW = dw.gamma5_matrix(V) @ D / (2 * kappa)
    w, vec = np.linalg.eigh(HW)
    return {
        "dense2": (L2, U2, dw.hopping_matrix(L2, U2)),
        "dense4": (L4, U4, dw.hopping_matrix(L4, U4)),
        "rough": ((4, 2, 2, 4), U4),
        "hw": (Lh, Uh, 1.5, HW, w, vec),
        "ov": ovpins.make_case(),
        "clover": ((4, 2, 2, 4), li.haar_links((4, 2, 2, 4), 41)),
    }


def battery(cases):
    yield lambda: pins.test_gamma_table_is_degrand_rossi_clifford()
    yield lambda: pins.test_free_field_plane_wave_closed_form((4, 6, 2, 8), True)
    yield lambda: pins.test_free_field_plane_wave_closed_form((6, 4, 4, 2), False)
    yield lambda: pins.test_gamma5_hermiticity_and_adjoint(cases["rough"])
    yield lambda: pins.test_gauge_covariance(cases["rough"])
    yield lambda: pins.test_mass_normalisation_and_hw_hermitian(cases["rough"])
    yield lambda: pins.test_dense_operator_matches(cases["dense2"])
    yield lambda: pins.test_dense_operator_matches(cases["dense4"])
    yield lambda: pins.test_dense_solve_matches_cg_eo(cases["dense2"])
    yield lambda: pins.test_dense_solve_matches_cg_eo(cases["dense4"])
    yield lambda: pins.test_chebyshev_scalar_error(0.01, 2.2e-13)
    yield lambda: pins.test_sign_function_matches_dense_sign(cases["hw"])
    yield lambda: ovpins.test_overlap_matches_dense_exact_sign(cases["ov"], 0.25)
    yield lambda: ovpins.test_overlap_ginsparg_wilson_and_normality(cases["ov"])
    yield lambda: ovpins.test_overlap_cg_matches_dense_solve(cases["ov"])
    yield lambda: ovpins.test_deflated_sign_is_exact_outside_the_window(cases["ov"])
    yield lambda: clpins.test_abelian_flux_closed_form(1, 2)
    yield lambda: clpins.test_clover_hermitian_chiral_blocks(cases["clover"])
    yield lambda: clpins.test_clover_gamma5_hermiticity_and_gauge_covariance(cases["clover"])
    yield lambda: clpins.test_clover_cg_matches_dense_solve((2, 2, 2, 2), 43)


def test_unmutated_battery_passes(small_cases, tmp_path, monkeypatch):
    mod = load_mutant(tmp_path, "none", "/*", "/*")
    monkeypatch.setattr(pins, "oracle", mod)
    monkeypatch.setattr(ovpins, "oracle", mod)
    monkeypatch.setattr(clpins, "oracle", mod)
    for check in battery(small_cases):
        check()


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutation(name, old, new, small_cases, tmp_path, monkeypatch):
    mod = load_mutant(tmp_path, name, old, new)
    monkeypatch.setattr(pins, "oracle", mod)
    monkeypatch.setattr(ovpins, "oracle", mod)
    monkeypatch.setattr(clpins, "oracle", mod)
    caught = []
    for i, check in enumerate(battery(small_cases)):
        try:
            check()
        except (AssertionError, np.linalg.LinAlgError, FloatingPointError, ValueError, ZeroDivisionError):
            caught.append(i)
            break
    assert caught, "no pin caught the planted mistake: %s" % name
