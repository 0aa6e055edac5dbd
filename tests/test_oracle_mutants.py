"""The pins catch plausible slips: each planted mistake below is compiled into
a copy of the oracle (on the CPU, in a temporary directory) and at least one
pin must fail against it.  The real oracle is untouched."""
from __future__ import annotations

import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lion_oracle.c")

MUTANTS = {
    "dc_sign_flipped": ("*ey = -a_rf * c * y + a_dc * y;\n    *ez = -2.0 * a_dc * z;",
                        "*ey = -a_rf * c * y + a_dc * y;\n    *ez = 2.0 * a_dc * z;"),
    "rf_y_sign_flipped": ("*ey = -a_rf * c * y + a_dc * y;", "*ey = a_rf * c * y + a_dc * y;"),
    "rf_term_dropped": ("*ex = a_rf * c * x + a_dc * x;", "*ex = a_dc * x;"),
    "pair_index_swapped": ("double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];\n            double r2 = dx * dx + dy * dy + dz * dz;\n            if (r2 == 0.0) {",
                           "double dx = x[j] - x[i], dy = y[i] - y[j], dz = z[i] - z[j];\n            double r2 = dx * dx + dy * dy + dz * dz;\n            if (r2 == 0.0) {"),
    "source_charge_is_target": ("double s = charge[j] *", "double s = charge[i] *"),
    "inverse_square_power": ("(1.0 / (r2 * sqrt(r2)))", "(1.0 / r2)"),
    "first_damping_dropped": ("            vx[i] = f * vx[i];\n            vy[i] = f * vy[i];\n            vz[i] = f * vz[i];\n            vx[i] = vx[i] + h * ax[i];",
                              "            vx[i] = vx[i] + h * ax[i];"),
    "force_time_not_advanced": ("double t = t_start + (double)(k + 1) * dt;", "double t = t_start + (double)k * dt;"),
    "full_kick": ("const double h = 0.5 * dt;", "const double h = dt;"),
    "coulomb_constant_2x": ("return 1.0 / (4.0 * OR_PI * OR_EPS0);", "return 1.0 / (2.0 * OR_PI * OR_EPS0);"),
    "self_term_kept_as_neighbour": ("if (j == i) continue;\n            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];\n            double r2 = dx * dx + dy * dy + dz * dz;\n            if (r2 == 0.0) {",
                                    "if (j == i + 1) continue;\n            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];\n            double r2 = dx * dx + dy * dy + dz * dz;\n            if (r2 == 0.0) {"),
    "free_ions_share_a_body": ("            if (body[i] >= 0 && body[j] == body[i]) continue;\n            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];\n            double r2 = dx * dx + dy * dy + dz * dz;\n            if (r2 == 0.0) {",
                               "            if (body[j] == body[i]) continue;\n            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];\n            double r2 = dx * dx + dy * dy + dz * dz;\n            if (r2 == 0.0) {"),
}

PINS = [
    lambda o: pins.test_accel_matches_40_digit_bruteforce(o, 3, 1),
    lambda o: pins.test_ten_steps_match_40_digit_bruteforce(o),
    lambda o: pins.test_single_ion_matches_transfer_matrices(o, "x"),
    lambda o: pins.test_single_ion_matches_transfer_matrices(o, "y"),
    lambda o: pins.test_two_ion_spacing_closed_form(o),
    lambda o: pins.test_laser_cooling_free_particle(o),
    lambda o: pins.test_body_exclusion_matches_40_digit_bruteforce(o),
    lambda o: pins.test_body_exclusion_special_cases(o),
]


COOLING_MUTANTS = {
    "beam_keeps_decayed_part": ("double d = (1.0 - fb) * (B->kx", "double d = fb * (B->kx"),
    "bath_variance_not_scaled": ("* (1.0 - c1 * c1));", ");"),
    "beam_ignores_species": ("if (B->gamma <= 0.0 || (B->species >= 0 && B->species != species)) continue;",
                             "if (B->gamma <= 0.0) continue;"),
    "philox_key_not_bumped": ("k0 += 0x9E3779B9u;", "k0 += 0u;"),
}

COOLING_PINS = [
    lambda o: pins.test_philox_known_answers(o),
    lambda o: pins.test_single_beam_cooling_free_ions(o),
    lambda o: pins.test_langevin_baths_follow_newtons_law_of_cooling(o),
]


def _build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found"
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(src.replace(old, new))  # the slip made wherever the text appears
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c99", "-shared", "-fPIC",
                    str(c), "-o", str(so), "-lm"], check=True)
    return str(so)


def _count_failures(so, pin_list):
    saved = oracle._lib
    oracle._lib = oracle.bind(so)
    failures = 0
    try:
        for pin in pin_list:
            try:
                pin(oracle)
            except (AssertionError, ValueError, FloatingPointError):
                failures += 1
    finally:
        oracle._lib = saved
    return failures


AVERAGE_MUTANTS = {
    "window_starts_one_step_early": ("const int64_t start = end - W + 1;",
                                     "const int64_t start = end - W;"),
    "mean_divides_by_w_minus_1": ("means[count * n + i] = acc / (double)W;",
                                  "means[count * n + i] = acc / (double)(W - 1);"),
    "windows_aligned_to_step_zero": ("const int64_t end = origin + m * W;",
                                     "const int64_t end = m * W;"),
}

AVERAGE_PINS = [
    lambda o: pins.test_time_average_of_damped_free_ion_closed_form(o),
    lambda o: pins.test_time_average_window_alignment(o),
]


RIGID_MUTANTS = {
    "torque_component_sign": ("T[3 * b] += o[1] * fz - o[2] * fy;",
                              "T[3 * b] += o[2] * fy - o[1] * fz;"),
    "full_angle_in_quaternion_step": ("quat_euler(q, w0, 0.5 * dt, qf);",
                                      "quat_euler(q, w0, dt, qf);"),
    "no_richardson_extrapolation": ("for (int k = 0; k < 4; ++k) r[k] = 2.0 * qh2[k] - qf[k];",
                                    "for (int k = 0; k < 4; ++k) r[k] = qf[k];"),
    "angular_momentum_not_damped": ("                L[3 * b + c] = f * L[3 * b + c];\n                V[3 * b + c] = V[3 * b + c] + h",
                                    "                V[3 * b + c] = V[3 * b + c] + h"),
    "body_frame_momentum_from_rows": ("p[k] = (A[k] * L[0] + A[3 + k] * L[1] + A[6 + k] * L[2]) * inv_i[k];",
                                      "p[k] = (A[3 * k] * L[0] + A[3 * k + 1] * L[1] + A[3 * k + 2] * L[2]) * inv_i[k];"),
    "member_velocity_without_spin": ("vx[i] = V[3 * b] + (w[1] * o[2] - w[2] * o[1]);",
                                     "vx[i] = V[3 * b];"),
    "force_not_mass_weighted": ("const double fx = mass[i] * ax[i], fy = mass[i] * ay[i], fz = mass[i] * az[i];",
                                "const double fx = ax[i], fy = ay[i], fz = az[i];"),
}

RIGID_PINS = [
    lambda o: pins.test_rigid_singleton_bodies_are_free_ions(o),
    lambda o: pins.test_rigid_body_com_follows_single_ion(o),
    lambda o: pins.test_rigid_rod_spin_is_uniform_rotation(o),
    lambda o: pins.test_rigid_asymmetric_top_converges_to_euler_equations(o),
    lambda o: pins.test_rigid_spin_down_under_damping(o),
    lambda o: pins.test_rigid_coulomb_explosion_conserves_momenta(o),
]


PSEUDO_MUTANTS = {
    "pseudo_strength_without_half": ("return (a_rf * a_rf) / (2.0 * tp->Omega * tp->Omega);",
                                     "return (a_rf * a_rf) / (tp->Omega * tp->Omega);"),
    "pseudo_dc_dropped": ("*ex = a_dc * x - k * x;", "*ex = -k * x;"),
    "pseudo_energy_sign": ("nsum_add(&d, 0.5 * charge[i] * (charge[i] / mass[i])",
                           "nsum_add(&d, -0.5 * charge[i] * (charge[i] / mass[i])"),
}

PSEUDO_PINS = [
    lambda o: pins.test_pseudo_trap_single_ion_is_harmonic(o, 40.0),
    lambda o: pins.test_pseudo_trap_single_ion_is_harmonic(o, 17.0),
    lambda o: pins.test_pseudo_energy_gradient_is_minus_force(o),
]


MINIMISER_MUTANTS = {
    "fmax_from_accelerations": ("if (sqrt(f2) > fm) fm = sqrt(f2);",
                                "if (sqrt(f2) / mass[i] > fm) fm = sqrt(f2) / mass[i];"),
    "step_cap_ignored": ("if (s > dmax) {", "if (s > 1e300 * dmax) {"),
    "velocity_against_force_kept": ("const double coef = (P > 0.0 && FF > 0.0) ? P / FF : 0.0;",
                                    "const double coef = (FF > 0.0) ? P / FF : 0.0;"),
}

MINIMISER_PINS = [
    lambda o: pins.test_minimised_chains_match_newton_roots(o, 3),
    lambda o: pins.test_minimiser_step_cap_and_projection(o),
]


HESSIAN_MUTANTS = {
    "hessian_dipole_sign": ("((a == b ? inv_r3 : 0.0) - 3.0 * r[a] * r[b] * inv_r5)",
                            "((a == b ? inv_r3 : 0.0) + 3.0 * r[a] * r[b] * inv_r5)"),
    "hessian_off_blocks_not_mass_weighted": ("D[(3 * i + a) * m + 3 * j + b] = h * w;",
                                             "D[(3 * i + a) * m + 3 * j + b] = h;"),
    "hessian_axial_trap_halved": ("diag[2][2] += 2.0 * charge[i] * a_dc;",
                                  "diag[2][2] += charge[i] * a_dc;"),
    "hessian_pseudo_not_species_scaled": ("diag[0][0] += charge[i] * qm * ps - charge[i] * a_dc;",
                                          "diag[0][0] += charge[i] * ps - charge[i] * a_dc;"),
}

HESSIAN_PINS = [
    lambda o: pins.test_normal_modes_of_one_ion(o, 40.0),
    lambda o: pins.test_normal_modes_of_one_ion(o, 17.0),
    lambda o: pins.test_normal_modes_of_minimised_chains(o, 3),
    lambda o: pins.test_hessian_is_minus_force_derivative(o),
]


@pytest.mark.parametrize("name", sorted(HESSIAN_MUTANTS))
def test_hessian_pins_reject_mutant(tmp_path, name, oracle_mod):
    so = _build_mutant(tmp_path, *HESSIAN_MUTANTS[name])
    assert _count_failures(so, HESSIAN_PINS) >= 1, f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(MINIMISER_MUTANTS))
def test_minimiser_pins_reject_mutant(tmp_path, name, oracle_mod):
    so = _build_mutant(tmp_path, *MINIMISER_MUTANTS[name])
    assert _count_failures(so, MINIMISER_PINS) >= 1, f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(PSEUDO_MUTANTS))
def test_pseudo_pins_reject_mutant(tmp_path, name, oracle_mod):
    so = _build_mutant(tmp_path, *PSEUDO_MUTANTS[name])
    assert _count_failures(so, PSEUDO_PINS) >= 1, f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(RIGID_MUTANTS))
def test_rigid_pins_reject_mutant(tmp_path, name, oracle_mod):
    so = _build_mutant(tmp_path, *RIGID_MUTANTS[name])
    assert _count_failures(so, RIGID_PINS) >= 1, f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(AVERAGE_MUTANTS))
def test_time_average_pins_reject_mutant(tmp_path, name, oracle_mod):
    so = _build_mutant(tmp_path, *AVERAGE_MUTANTS[name])
    assert _count_failures(so, AVERAGE_PINS) >= 1, f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(COOLING_MUTANTS))
def test_cooling_pins_reject_mutant(tmp_path, name, oracle_mod):
    so = _build_mutant(tmp_path, *COOLING_MUTANTS[name])
    assert _count_failures(so, COOLING_PINS) >= 1, f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name, oracle_mod):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(old, new)  # the slip made wherever the text appears
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c99", "-shared", "-fPIC",
                    str(c), "-o", str(so), "-lm"], check=True)
    saved = oracle._lib
    oracle._lib = oracle.bind(str(so))
    failures = 0
    try:
        for pin in PINS:
            try:
                pin(oracle)
            except (AssertionError, ValueError, FloatingPointError):
                failures += 1
    finally:
        oracle._lib = saved
    assert failures >= 1, f"no pin caught mutant {name}"
