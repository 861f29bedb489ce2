"""The pins have teeth: plant plausible mistakes in a copy of the oracle
source, build it on the CPU, and check that the pins reject every mutant."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import build as obuild
from tests import closed_form as cf
from tests import test_oracle_mc9_pins as mc9_pins
from tests import test_oracle_mg_pins as mg_pins
from tests import test_oracle_rb3_pins as rb3_pins
from tests import test_oracle_pins as pins

MUTANTS = {
    "dropped_left_neighbour": ("s = s + AT(u, i, j - 1);\n            double t = h2", "double t = h2"),
    "wrong_sign_of_f": ("s = s - t;\n            AT(u, i, j) = 0.25 * s;", "s = s + t;\n            AT(u, i, j) = 0.25 * s;"),
    "wrong_index_up": ("double s = AT(u, i + 1, j) + AT(u, i - 1, j);\n            s = s + AT(u, i, j + 1);\n            s = s + AT(u, i, j - 1);\n            double t = h2 * AT(f, i, j);\n            s = s - t;\n            AT(u, i, j) = 0.25 * s;",
                       "double s = AT(u, i + 1, j) + AT(u, i + 1, j);\n            s = s + AT(u, i, j + 1);\n            s = s + AT(u, i, j - 1);\n            double t = h2 * AT(f, i, j);\n            s = s - t;\n            AT(u, i, j) = 0.25 * s;"),
    "colours_swapped": ("(i % 2 == 0) ? (colour == 0 ? 2 : 1) : (colour == 0 ? 1 : 2);\n        for (int64_t j = j_start; j <= n; j += 2) {\n            double",
                        "(i % 2 == 0) ? (colour == 0 ? 1 : 2) : (colour == 0 ? 2 : 1);\n        for (int64_t j = j_start; j <= n; j += 2) {\n            double"),
    "black_before_red": ("rbgs_ref_half_sweep_f64(n, ld, h, u, f, 0);\n        rbgs_ref_half_sweep_f64(n, ld, h, u, f, 1);",
                         "rbgs_ref_half_sweep_f64(n, ld, h, u, f, 1);\n        rbgs_ref_half_sweep_f64(n, ld, h, u, f, 0);"),
    # the binary32 residual sums its neighbours in binary32 (the widening dropped)
    "residual_f32_not_widened": ("double s = (double)AT(u, i + 1, j) + (double)AT(u, i - 1, j);",
                                 "double s = AT(u, i + 1, j) + AT(u, i - 1, j);"),
    "residual_missing_centre": ("double lap = (s - 4.0 * (double)AT(u, i, j)) * inv_h2;",
                                "double lap = (s - 2.0 * (double)AT(u, i, j)) * inv_h2;"),
    "h_not_squared": ("const double h2 = h * h;\n#pragma omp parallel for schedule(static)\n    for (int64_t i = 1; i <= n; ++i) {\n        /* red",
                      "const double h2 = h;\n#pragma omp parallel for schedule(static)\n    for (int64_t i = 1; i <= n; ++i) {\n        /* red"),
    # multigrid cycle
    "mg_correction_subtracted": ("AT(u, i, j) = AT(u, i, j) + v;", "AT(u, i, j) = AT(u, i, j) - v;"),
    "mg_coarse_h_not_doubled": ("lv[l].h = l == 0 ? h : 2.0 * lv[l - 1].h;",
                                "lv[l].h = l == 0 ? h : lv[l - 1].h;"),
    "mg_full_weighting_centre": ("((row[0] + 2.0 * row[1]) + row[2]) * 0.0625",
                                 "((row[0] + row[1]) + row[2]) * 0.0625"),
    "mg_restrict_column_shift": ("2.0 * AT(r, i, 2 * J)) + AT(r, i, 2 * J + 1);",
                                 "2.0 * AT(r, i, 2 * J)) + AT(r, i, 2 * J - 1);"),
    "mg_prolong_corner_weight": ("(EC(I + 1, J) + EC(I + 1, J + 1))) * 0.25;",
                                 "(EC(I + 1, J) + EC(I + 1, J + 1))) * 0.5;"),
    "mg_prolong_row_shift": ("v = (EC(I, J) + EC(I + 1, J)) * 0.5;",
                             "v = (EC(I, J) + EC(I - 1, J)) * 0.5;"),
    "mg_postsmoothing_dropped": ("rbgs_ref_sweep_f64(a->n, a->ld, a->h, a->u, a->f, nu2);",
                                 "rbgs_ref_sweep_f64(a->n, a->ld, a->h, a->u, a->f, 0);"),
    # 4-colour 9-point Gauss-Seidel
    "mc9_dropped_corner": ("c = c + AT(u, i - 1, j - 1);\n            double s = 4.0 * e + c;",
                           "double s = 4.0 * e + c;"),
    "mc9_edge_weight": ("double s = 4.0 * e + c;", "double s = 2.0 * e + c;"),
    "mc9_divisor": ("AT(u, i, j) = s / 20.0;", "AT(u, i, j) = s / 16.0;"),
    "mc9_h_scale": ("const double c6 = 6.0 * (h * h);", "const double c6 = 4.0 * (h * h);"),
    "mc9_colour_order": ("for (int32_t colour = 0; colour < 4; ++colour)\n            rbgs_ref_mc9_quarter_sweep_f64",
                         "for (int32_t colour = 3; colour >= 0; --colour)\n            rbgs_ref_mc9_quarter_sweep_f64"),
    "rb3_dropped_k_minus": ("s = s + AT3(u, i, j, k - 1);\n                const double t = h2",
                            "const double t = h2"),
    "rb3_divisor": ("AT3(u, i, j, k) = s / 6.0;", "AT3(u, i, j, k) = s / 4.0;"),
    "rb3_colour_parity": ("const int64_t k0 = ((i + j + 1) & 1) == colour ? 1 : 2;",
                          "const int64_t k0 = ((i + j) & 1) == colour ? 1 : 2;"),
    "rb3_wrong_plane": ("double s = AT3(u, i + 1, j, k) + AT3(u, i - 1, j, k);\n                s = s + AT3(u, i, j + 1, k);\n                s = s + AT3(u, i, j - 1, k);\n                s = s + AT3(u, i, j, k + 1);\n                s = s + AT3(u, i, j, k - 1);\n                const double t",
                        "double s = AT3(u, i + 1, j, k) + AT3(u, i + 1, j, k);\n                s = s + AT3(u, i, j + 1, k);\n                s = s + AT3(u, i, j - 1, k);\n                s = s + AT3(u, i, j, k + 1);\n                s = s + AT3(u, i, j, k - 1);\n                const double t"),
    "mc9_colour_parity": ("const int64_t i0 = (colour & 1) ? 1 : 2, j0 = (colour & 2) ? 1 : 2;",
                          "const int64_t i0 = (colour & 2) ? 1 : 2, j0 = (colour & 1) ? 1 : 2;"),
}


def _build_mutant(tmp_path, name):
    src = open(obuild.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new, 1)
    path = os.path.join(str(tmp_path), f"rbgs_{name}.c")
    lib = os.path.join(str(tmp_path), f"lib_{name}.so")
    with open(path, "w") as fh:
        fh.write(mutated)
    subprocess.run(["gcc", *obuild.CFLAGS, path, "-o", lib, "-lm"], check=True)
    return lib


def _pins_that_run():
    """A small set of pins; a mutant must fail at least one."""
    yield lambda: pins.test_half_sweep_visits_exactly_algorithm1_points(oracle)
    yield lambda: pins.test_n1_single_point(oracle)
    yield lambda: pins.test_single_mode_iterate(oracle, 15, 40)
    yield lambda: pins.test_multi_mode_iterate(oracle)
    yield lambda: pins.test_converges_to_dense_solve(oracle, 9)
    yield lambda: pins.test_residual_special_cases(oracle)
    yield lambda: pins.test_residual_f32_is_fp64_residual_of_widened_iterate(oracle)
    yield lambda: mg_pins.test_restrict_constant_and_bilinear(oracle, 3)
    yield lambda: mg_pins.test_prolong_bilinear_exact_and_additive(oracle, 3)
    yield lambda: mg_pins.test_restrict_is_quarter_adjoint_of_prolong(oracle)
    yield lambda: mg_pins.test_converges_to_dense_solve(oracle, 15, (1, 1))
    yield lambda: mg_pins.test_vcycle_factor_is_textbook_and_h_independent(oracle, 63)
    yield lambda: mc9_pins.test_quarter_sweep_touches_exactly_its_colour(oracle)
    yield lambda: mc9_pins.test_one_point(oracle)
    yield lambda: mc9_pins.test_converges_to_dense_solve(oracle, 7)
    yield lambda: mc9_pins.test_updated_colour_has_zero_residual(oracle)
    yield lambda: rb3_pins.test_half_sweep_touches_exactly_its_colour(oracle)
    yield lambda: rb3_pins.test_one_point(oracle)
    yield lambda: rb3_pins.test_converges_to_dense_solve(oracle, 4)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name):
    lib = _build_mutant(tmp_path, name)
    caught = 0
    with oracle.use_library(lib):
        for pin in _pins_that_run():
            try:
                pin()
            except AssertionError:
                caught += 1
    assert caught >= 1, f"mutant {name} passed every pin"


def test_unmutated_source_passes(tmp_path):
    src_copy = os.path.join(str(tmp_path), "lib_clean.so")
    subprocess.run(["gcc", *obuild.CFLAGS, obuild.SRC, "-o", src_copy, "-lm"], check=True)
    with oracle.use_library(src_copy):
        for pin in _pins_that_run():
            pin()


# --------------------------------------------------------------------------
# The reference network's Adam (oracle/unet_ref.py): planted mistakes in a
# copy of its source, loaded as a separate module, must fail the Adam pins.
# --------------------------------------------------------------------------
PY_MUTANTS = {
    "adam_bias_exponent_fixed": ("mh = m / (1 - beta1 ** t)", "mh = m / (1 - beta1)"),
    "adam_v_uncorrected": ("vh = v / (1 - beta2 ** t)", "vh = v"),
    "adam_betas_swapped": ("m[...] = beta1 * m + (1 - beta1) * g[k]\n        v[...] = beta2 * v + (1 - beta2) * g[k] * g[k]",
                           "m[...] = beta2 * m + (1 - beta2) * g[k]\n        v[...] = beta1 * v + (1 - beta1) * g[k] * g[k]"),
    "adam_step_counter_late": ("state[\"t\"] = state.get(\"t\", 0) + 1\n    t = state[\"t\"]",
                               "t = state.get(\"t\", 0) + 1\n    state[\"t\"] = max(1, t - 1)"),
    "adam_eps_inside_sqrt": ("np.sqrt(vh) + eps", "np.sqrt(vh + eps)"),
}


def _load_py_mutant(name):
    import importlib.util
    import types
    from oracle import unet_ref
    src = open(unet_ref.__file__).read()
    old, new = PY_MUTANTS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType(f"unet_ref_{name}")
    mod.__file__ = unet_ref.__file__
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    assert importlib.util is not None
    return mod


def _adam_pins():
    from tests import test_unet_ref as ur
    return [ur.check_adam_first_step, ur.check_adam_constant_gradient, ur.check_adam_sum_form]


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_adam_pins_reject_mutant(name):
    mod = _load_py_mutant(name)
    caught = 0
    for pin in _adam_pins():
        try:
            pin(mod)
        except AssertionError:
            caught += 1
    assert caught >= 1, f"mutant {name} passed every Adam pin"


def test_adam_pins_pass_unmutated_source():
    from oracle import unet_ref
    for pin in _adam_pins():
        pin(unet_ref)
