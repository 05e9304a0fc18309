"""The oracle's pins catch one-term mistakes.

Each case plants one plausible mistake in a copy of oracle/qtraj_oracle.c (a
flipped sign, a wrong coefficient, a shifted index, a changed comparison),
builds that copy, and runs the pin tests that should catch it against it in
a child process (QTO_LIB).  The case passes when those pins FAIL on the
mutant.  Nothing here touches the real oracle or the GPU library."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "qtraj_oracle.c")

P = "tests/test_oracle_pins.py::"
C = "tests/test_oracle_closed_forms.py::"
MUNICH = C + "test_munich_potential_phase_closed_form"
KSU = C + "test_ksu_potential_phase_closed_form"

# (name, original text, mutated text, pin tests that must fail)
MUTATIONS = [
    ("octet_coulomb_sign", "*VR = alpha / (8.0 * r)", "*VR = -alpha / (8.0 * r)", [MUNICH]),
    ("octet_coulomb_1_8", "*VR = alpha / (8.0 * r)", "*VR = alpha / (9.0 * r)", [MUNICH]),
    ("singlet_coulomb_sign", "*VR = -alpha / r", "*VR = alpha / r", [MUNICH]),
    ("singlet_gamma_half", "0.5 * gamma * r * r", "0.25 * gamma * r * r", [MUNICH]),
    ("octet_gamma_7_32", "(7.0 / 32.0) * gamma", "(7.0 / 16.0) * gamma", [MUNICH]),
    ("octet_kappa_7_32", "-(7.0 / 32.0) * kappa", "-(7.0 / 16.0) * kappa", [MUNICH]),
    ("singlet_kappa_half", "*VI = -0.5 * kappa", "*VI = -0.25 * kappa", [MUNICH]),
    ("centrifugal_l_squared", "double centrifugal = (double)l * (double)(l + 1)",
     "double centrifugal = (double)l * (double)l", [MUNICH]),
    ("alpha_c_f", "(4.0 / 3.0) * p->alpha_s; }", "(3.0 / 4.0) * p->alpha_s; }", [MUNICH]),
    ("kappa_fit_coefficient", "0.00397, -0.08341, 0.98031", "0.00397, -0.08341, 0.98013",
     [C + "test_kappa_hat_fits_printed_coefficients"]),
    ("temperature_step_not_linear", "return tt->T[i] + (tt->T[i + 1] - tt->T[i]) * w;",
     "return tt->T[i];", [MUNICH]),
    ("ksu_no_string_breaking", "(kms <= vsb ? kms : vsb)", "kms", [KSU]),
    ("ksu_sigma_term_sign", "- KSU_SIGMA * r * e;", "+ KSU_SIGMA * r * e;", [KSU]),
    ("ksu_centrifugal_missing", "*VR = (kms <= vsb ? kms : vsb) + (double)l * (double)(l + 1)",
     "*VR = (kms <= vsb ? kms : vsb) + 0.0 * (double)(l + 1)", [KSU]),
    ("steps_strict_T_final", "if (qto_temperature(tt, t) < tt->T_final) break;",
     "if (qto_temperature(tt, t) <= tt->T_final) break;", [C + "test_num_steps_by_hand"]),
    ("steps_table_end", "if (t > tt->tau[tt->n - 1]) break;", "if (t >= tt->tau[tt->n - 1]) break;",
     [C + "test_num_steps_by_hand"]),
    ("mean_radius_index", "num += (double)j * dr * w2;", "num += (double)(j + 1) * dr * w2;",
     [C + "test_mean_radius_exact_cases"]),
    ("survival_floor_dropped", "(s->init_overlap[bb] > 1e-12)", "(s->init_overlap[bb] > 0.0)",
     [C + "test_survival_of_a_barely_populated_state"]),
    ("dst_scale", "double scale = sqrt(2.0 / (double)N);", "double scale = sqrt(2.0 / (double)(N - 1));",
     [P + "test_dst_matches_scipy_and_is_involution"]),
    ("kinetic_reduced_mass", "return pk * pk / p->mass;", "return pk * pk / (2.0 * p->mass);",
     [P + "test_sine_mode_phase", P + "test_coulomb_eigenstate_is_stationary"]),
    ("half_step_modulus", "double modulus = exp(0.5 * p->dt * VI);", "double modulus = exp(p->dt * VI);",
     [P + "test_width_decay_without_kinetic_term"]),
    ("octet_to_singlet_2_7", "if (u_c < 2.0 / 7.0) *c = QTO_SINGLET;", "if (u_c < 5.0 / 7.0) *c = QTO_SINGLET;",
     [P + "test_jump_rule_matches_printed_probabilities"]),
    ("l_down_probability", "double p_down = (double)(*l) / (double)(2 * (*l) + 1);",
     "double p_down = (double)(*l + 1) / (double)(2 * (*l) + 1);",
     [P + "test_jump_rule_matches_printed_probabilities"]),
    ("jump_multiplies_by_r", "double rj = (double)j * dr;", "double rj = (double)(j + 1) * dr;",
     [P + "test_jump_multiplies_by_r_and_renormalises"]),
    ("jump_at_equality", "if (norm <= r) {", "if (norm < r - 1e-3) {",
     [P + "test_waiting_time_rule_and_renormalisation"]),
]


@pytest.mark.parametrize("name,orig,mut,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_the_mutation(tmp_path, name, orig, mut, pins):
    src = open(SRC).read()
    assert src.count(orig) >= 1, "mutation %s: text not found" % name
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(orig, mut, 1))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
                    "-ffp-contract=off", "-I" + os.path.join(ROOT, "oracle"), str(mutant), "-o",
                    lib, "-lm"], check=True)
    env = dict(os.environ, QTO_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + pins,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, "mutation %s survived its pins:\n%s" % (name, r.stdout[-2000:])
