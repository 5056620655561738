"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of oracle/oracle.c (a dropped
term, a wrong sign, index or constant, a swapped rule), builds that copy with
the same compiler line as the real oracle, and runs the pins that should catch
it against the copy (ORACLE_LIB_PATH).  The case passes only if at least one of
those pins fails.  The text each mutation replaces must occur exactly once in
the oracle, so the cases follow the oracle as it changes.

This is CPU-only test infrastructure; nothing runs on the GPU.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = "tests/test_oracle_pins.py::"
RULES = "tests/test_oracle_pcg_rules.py::"

# name -> ([(original text, planted text), ...], [pins expected to catch it])
MUTANTS = {
    "w_ij multiplies psi_j (as printed) instead of psi_i": (
        [("P->Gdd[i][j] * phr[j * N + x]) * si[x];", "P->Gdd[i][j] * phr[j * N + x]) * psi[j * N + x];")],
        [PINS + "test_model_w_ij_uses_psi_i", PINS + "test_model_coefficients_are_geodesic_derivatives"]),
    "sign of the coupling term in the LHY ratio": (
        [("(e11 * delta + 2.0 * e12 * e21 * n2) / s", "(e11 * delta - 2.0 * e12 * e21 * n2) / s")],
        [PINS + "test_lhy_homogeneity_euler_and_fd", PINS + "test_lhy_component_swap_symmetry"]),
    "kinetic multiplier |k|^2 without the 1/2": (
        [("g->K2h[i] = 0.5 * k2;", "g->K2h[i] = k2;")],
        [PINS + "test_plane_wave_is_kinetic_eigenfunction", PINS + "test_gaussian_kinetic_energy_closed_form"]),
    "kx in place of kz in the dipolar kernel": (
        [("else g->Ud[i] = (3.0 * kz * kz / k2 - 1.0)", "else g->Ud[i] = (3.0 * kx * kx / k2 - 1.0)")],
        [PINS + "test_dipolar_energy_of_cylindrical_gaussian"]),
    "component index in n_2''": (
        [("n2pp = p2 - n2 * gam2inv[1];", "n2pp = p2 - n2 * gam2inv[0];")],
        [PINS + "test_model_coefficients_are_geodesic_derivatives"]),
    "eta_21 in place of eta_12 in the LHY couplings": (
        [("double e12 = P->G[0][1] + P->Gdd[0][1] * a;\n        double e21 = P->G[1][0] + P->Gdd[1][0] * a;\n"
          "        double delta = e11 * n1 - e22 * n2;\n        double s = sqrt(",
          "double e12 = P->G[1][0] + P->Gdd[1][0] * a;\n        double e21 = P->G[1][0] + P->Gdd[1][0] * a;\n"
          "        double delta = e11 * n1 - e22 * n2;\n        double s = sqrt(")],
        [PINS + "test_lhy_without_dipoles_is_u_independent_closed_form"]),
    "omega in place of omega^2 in the trap": (
        [("0.5 * (P->omega[0] * P->omega[0] * x * x +", "0.5 * (P->omega[0] * x * x +")],
        [PINS + "test_trap_energy_closed_form"]),
    "index of the parameter derivative dV/d eta_12": (
        [("dv[1] = sq > 0.0 ? sg * 2.0 * e21 * n1 * n2 / sq : 0.0;",
          "dv[1] = sq > 0.0 ? sg * 2.0 * e12 * n1 * n2 / sq : 0.0;")],
        [PINS + "test_param_grad_matches_finite_differences"]),
    "HS+ and PR+ denominators swapped": (
        [("den += w[i] * dV * (o->beta == 1 ? 0.0 : yp);", "den += w[i] * dV * (o->beta == 0 ? 0.0 : yp);"),
         ("if (o->beta == 1) den = rz_old;", "if (o->beta == 0) den = rz_old;")],
        [RULES + "test_hs_plus_direction_is_conjugate_to_the_residual_change", RULES + "test_pr_plus_ratio"]),
    "stacked-product weights (N_i/N)^2 dropped": (
        [("const double w[2] = { (P->N[0] / (P->N[0] + P->N[1])) * (P->N[0] / (P->N[0] + P->N[1])),\n"
          "                          (P->N[1] / (P->N[0] + P->N[1])) * (P->N[1] / (P->N[0] + P->N[1])) };",
          "const double w[2] = { 1.0, 1.0 };")],
        [RULES + "test_hs_plus_direction_is_conjugate_to_the_residual_change", RULES + "test_pr_plus_ratio"]),
    "negative beta used (no max(., 0))": (
        [("            if (beta < 0.0) beta = 0.0;\n            beta_num = num;", "            beta_num = num;"),
         ("int level = (beta > 0.0) ? 0 : 1;", "int level = (beta != 0.0) ? 0 : 1;")],
        [RULES + "test_beta_is_clipped_at_zero"]),
    "Armijo sufficient-decrease term with the wrong sign": (
        [("Et <= cur.t.E + o->armijo_c1 * alpha * m.E1 + tau", "Et <= cur.t.E - o->armijo_c1 * alpha * m.E1 + tau")],
        [RULES + "test_armijo_halving_along_the_exact_geodesic"]),
    "backtracking factor other than 1/2": (
        [("alpha *= 0.5;", "alpha *= 0.6;")],
        [RULES + "test_armijo_halving_along_the_exact_geodesic"]),
    "restart period ignored": (
        [("(o->restart_period > 0 && n % o->restart_period == 0)", "(o->restart_period > 0 && 0)")],
        [RULES + "test_restart_period"]),
    "tangent projection of the direction dropped": (
        [("for (long x = 0; x < N; ++x) p[i * N + x] -= c * psi[i * N + x];", "(void)c;")],
        [RULES + "test_direction_is_projected_minus_z_plus_beta_p_old"]),
    "theta_max clamp of the step dropped": (
        [("if (alpha * pmax > o->theta_max) alpha = o->theta_max / pmax;", "")],
        [RULES + "test_model_step_minimises_the_quadratic_model"]),
    "composite fallback to P_Delta instead of P_V": (
        [("if (level == 2) precond_apply(&g, P, &cur, 1, o->sigma, 0.0, r, z);",
          "if (level == 2) precond_apply(&g, P, &cur, 2, o->sigma, 0.0, r, z);")],
        [RULES + "test_composite_fallback_ladder"]),
    "stall reference reset without halving": (
        [("if (res_max < 0.5 * stall_ref) {", "if (res_max < 0.9 * stall_ref) {")],
        [RULES + "test_stall_stop_fires_at_the_first_step_its_definition_names"]),
    "slab cut: sign of the sin term": (
        [("(kr2 * cos(kz * Z) - kr * kz * sin(kz * Z))", "(kr2 * cos(kz * Z) + kr * kz * sin(kz * Z))")],
        ["tests/test_oracle_slab_dipoles.py::test_layer_energy_closed_form"]),
    "slab cut: zero mode 0 instead of 2": (
        [("if (k2 == 0.0) return 2.0;", "if (k2 == 0.0) return 0.0;")],
        ["tests/test_oracle_slab_dipoles.py::test_layer_energy_closed_form"]),
    "blend: the weight applied to P_Delta": (
        [("z[i * N + x] = w * zv[i * N + x] + (1.0 - w) * z[i * N + x];",
          "z[i * N + x] = (1.0 - w) * zv[i * N + x] + w * z[i * N + x];")],
        [PINS + "test_blended_preconditioner_end_weights_symmetry_positivity"]),
    "blend: adaptive weight from the kinetic share": (
        [("return (Pot + K > 0.0) ? Pot / (Pot + K) : 0.5;", "return (Pot + K > 0.0) ? K / (Pot + K) : 0.5;")],
        [PINS + "test_blended_preconditioner_on_plane_waves"]),
    "root-split rule: map without the sine factor in the weights": (
        [("w[k * n + j] = tw[j] * (q - p) * 0.5 * M_PI * sin(M_PI * t[j]);",
          "w[k * n + j] = tw[j] * (q - p);")],
        ["tests/test_oracle_lhy_rule.py::test_single_component_matches_closed_form"]),
    "failed line search not retried with beta = 0": (
        [("if (level == 0) { level = 1; rep->n_restarts++; path |= 2; continue; }", "")],
        [RULES + "test_beta_zero_retry_after_a_failed_line_search"]),
}


def _plant(src, edits):
    for old, new in edits:
        assert src.count(old) == 1, f"mutation site not unique or missing: {old[:60]!r}"
        src = src.replace(old, new)
    return src


def _run_mutant(name, tmpdir):
    edits, pins = MUTANTS[name]
    src = _plant(open(SRC).read(), edits)
    tag = f"m{sorted(MUTANTS).index(name)}"
    c_path = os.path.join(tmpdir, f"{tag}.c")
    so_path = os.path.join(tmpdir, f"lib{tag}.so")
    with open(c_path, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-w", c_path, "-o", so_path, "-lm"],
                   check=True)
    env = dict(os.environ, ORACLE_LIB_PATH=so_path, OMP_NUM_THREADS="2", PYTHONPATH=ROOT)
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return p.returncode, p.stdout[-2000:]


@pytest.fixture(scope="module")
def mutant_results(tmp_path_factory):
    tmpdir = str(tmp_path_factory.mktemp("mutants"))
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(_run_mutant, name, tmpdir) for name in MUTANTS}
        return {name: f.result() for name, f in futs.items()}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_fails_a_pin(mutant_results, name):
    rc, out = mutant_results[name]
    # exit status 1: the pins ran and at least one failed (2-5 would be an error or no tests)
    assert rc == 1, f"{name}: pins did not catch it (rc={rc})\n{out}"
