"""The pins catch planted mistakes.

Each case copies oracle/homg_oracle.c, plants one plausible mistake by text
substitution, builds the copy with gcc into a temporary library, points the
oracle at it and runs a few pins from test_oracle_pins: at least one must
fail.  Everything runs on the CPU; the real oracle is restored afterwards.
"""
import os
import subprocess

import pytest

import test_oracle_pins as P  # noqa: E402  (tests/ is on sys.path under pytest)
from oracle import homg as O

SRC = os.path.join(os.path.dirname(O.__file__), "homg_oracle.c")

MUTANTS = {
    "relax_sign": ("hl * hl * rv - flux", "hl * hl * rv + flux"),
    "relax_spacing": ("const double hl = (double)l / (double)(n - 1);", "const double hl = 1.0 / (double)(n - 1);"),
    "relax_stride": ("neighbours(d, l, off);\n    size_t p", "neighbours(d, 1, off);\n    size_t p"),
    "fw_weight": ("double w = (ox == 0 ? 0.5 : 0.25) * (oy == 0 ? 0.5 : 0.25);",
                  "double w = (ox == 0 ? 0.5 : 0.25) * (oy == 0 ? 0.25 : 0.5);"),
    "fw_offset": ("s += w * rf[node(nf, kf, 2 * J + oy, 2 * I + ox)];", "s += w * rf[node(nf, kf, 2 * J + oy, 2 * I + 2 * ox)];"),
    "interp_weight": ("double w = (bx ? ti : 1.0 - ti) * (by ? tj : 1.0 - tj);",
                      "double w = (bx ? 1.0 - ti : ti) * (by ? tj : 1.0 - tj);"),
    "interp_no_delay": ("e_new[p] = oracle_interpolate(d, n, m, e_old, k, j, i);",
                        "e_new[p] = oracle_interpolate(d, n, m, e_new, k, j, i);"),
    "residual_sign": ("r[p] = f[p] - au * inv_h2;", "r[p] = f[p] + au * inv_h2;"),
    "residual_drop_h2": ("r[p] = f[p] - au * inv_h2;", "r[p] = f[p] - au;"),
    "relax_drop_neighbour": ("for (int t = 0; t < 2 * d; ++t) {\n        size_t q = node(n, k + off[t][0], j + off[t][1], i + off[t][2]);\n        double apq",
                             "for (int t = 1; t < 2 * d; ++t) {\n        size_t q = node(n, k + off[t][0], j + off[t][1], i + off[t][2]);\n        double apq"),
    "face_arith_mean": ("return 2.0 * a[p] * a[q] / (a[p] + a[q]);", "return 0.5 * (a[p] + a[q]);"),
}


def _pins():
    yield lambda: P.test_A_symmetric(2, 17, True)
    yield lambda: P.test_A_eigenpairs(2, 33, (3, 7))
    yield lambda: P.test_residual_matches_dense_assembly(2, 9)
    yield lambda: P.test_homg_converges_to_dense_lu(2, 17)
    yield lambda: P.test_full_weighting_of_sine_mode(2, 33, (5, 11))
    yield lambda: P.test_full_weighting_adjoint_of_interpolation(2, 17)
    yield lambda: P.test_interpolation_reproduces_multilinear(2, 33, 3)
    yield lambda: P.test_jacobi_damps_eigenmode_by_its_factor(2, 65, 2, (1, 6))
    yield lambda: P.test_level_relaxation_fixed_point_is_level_system(2, 33, 1, True)
    yield lambda: P.test_lattice_independence_identity(2, 33, 4)
    yield P.test_fig3_spike_then_pyramid


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / ("libmut_%s.so" % name)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    str(mut), "-o", str(so), "-lm"], check=True)
    saved = O._lib
    O._lib = O.load_library(str(so))
    caught = []
    try:
        for pin in _pins():
            try:
                pin()
            except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError, IndexError):
                caught.append(pin)
    finally:
        O._lib = saved
    assert caught, "no pin caught mutant " + name
