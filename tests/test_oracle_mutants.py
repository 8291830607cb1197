"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch each one: the pins must not be blind to a dropped term,
a wrong sign, a swapped index or a transposed operand."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "sdd_oracle.c")

PINS = "test_oracle_pins.py"
KPINS = "test_kappa_pins.py"
KAPPA_SECTION = "Discontinuous kappa: the interface scheme"

# the two branches of an interface step's time split (resume on side i, on side j)
KAPPA_SPLIT = ("            T[si] += dt - 0.5 * (dt - tg) * pi_;\n            T[sj] += 0.5 * (dt - tg) * pi_;\n"
               "        } else {                                         /* resume on side j */\n"
               "            cy = P->y_if + towards * h;\n"
               "            T[si] += tg + 0.5 * (dt - tg) * pj;\n            T[sj] += 0.5 * (dt - tg) * (2.0 - pj);")

# (name, original text, mutated text, pins expected to fail[, pin file])
MUTANTS = [
    ("no_bridge", "if (q <= P->dt * L) {", "if (0) {", ["test_mean_exit_time_series"]),
    ("phase_sign", "out->w_im = g[1] * cs - g[0] * sn;", "out->w_im = g[1] * cs + g[0] * sn;",
     ["test_plane_wave_unit_square"]),
    ("phase_rate_factor", "c[P->n_regions] = alpha_of_sigma(P, P->sigma_background) * P->dt / 2.0;",
     "c[P->n_regions] = alpha_of_sigma(P, P->sigma_background) * P->dt;", ["test_plane_wave_unit_square"]),
    ("walls_swapped", "wall = upper[0] ? 1 : 3;", "wall = upper[0] ? 3 : 1;", ["test_linear_harmonic_alpha_zero"]),
    ("tangent_transposed", "t = z + fr * (zn - z);", "t = y + fr * (yn - y);", ["test_linear_harmonic_alpha_zero"]),
    ("bridge_factor", "double q = (2.0 * d0) * d1;", "double q = d0 * d1;", ["test_mean_exit_time_series"]),
    ("normals_reused", "orc_box_muller(orc_u01(w[2]), orc_u01(w[3]), out);",
     "orc_box_muller(orc_u01(w[0]), orc_u01(w[1]), out);", ["test_mean_exit_time_series"]),
    ("partial_phase_dropped", "S += c[orc_region(P, y, z)] * fr;", "S += 0.0 * fr;",
     ["test_single_step_crossing_by_hand"]),
    ("phase_start_point", "S += c[orc_region(P, yn, zn)];", "S += c[orc_region(P, y, z)];",
     ["test_discrete_scheme_exact_on_a_strip"]),
    ("table_index_shift", "out[0] = (1.0 - lam) * gw[2 * i] + lam * gw[2 * i + 2];",
     "out[0] = (1.0 - lam) * gw[2 * i + 2] + lam * gw[2 * i + 4];", ["test_table_interpolation_linear_exact"]),
    ("air_phase", "if (P->freq_hz > 0.0) {", "if (sigma == 0.0) return P->alpha_direct;\n    if (P->freq_hz > 0.0) {",
     ["test_layered_halfspace_is_1d"]),
    ("mu0_without_pi", "double mu0 = 4.0e-7 * pi;", "double mu0 = 4.0e-7;", ["test_frequency_branch_skin_depth"]),
    ("frequency_for_omega", "double omega = 2.0 * pi * P->freq_hz;", "double omega = P->freq_hz;",
     ["test_frequency_branch_skin_depth"]),
    ("length_unit_not_squared", "return omega * mu0 * sigma * (L * L);", "return omega * mu0 * sigma * L;",
     ["test_frequency_branch_skin_depth"]),
    ("region_order", "for (int r = 0; r < P->n_regions; ++r)\n        if (in_primitive",
     "for (int r = P->n_regions - 1; r >= 0; --r)\n        if (in_primitive", ["test_region_predicate"]),
    # the discontinuous-kappa walk
    ("kappa_p_swapped", "double pi_ = ki / (ki + kj), pj = 1.0 - pi_;", "double pi_ = kj / (ki + kj), pj = 1.0 - pi_;",
     ["test_piecewise_linear_harmonic_is_unbiased"], KPINS),
    ("kappa_side_flipped", "double towards = (si == 0) ? 1.0 : -1.0;", "double towards = (si == 0) ? -1.0 : 1.0;",
     ["test_piecewise_linear_harmonic_is_unbiased"], KPINS),
    ("kappa_unequal_radii", "cy = P->y_if + towards * h;", "h = sqrt(kj * dt);\n            cy = P->y_if + towards * h;",
     ["test_piecewise_linear_harmonic_is_unbiased"], KPINS),
    ("kappa_printed_share", "T[sj] += 0.5 * (dt - tg) * (2.0 - pj);", "T[sj] += 0.5 * (dt - tg) * (1.0 + pj);",
     ["test_occupation_shares_sum_to_the_step"], KPINS),
    ("kappa_rates_swapped", "double ei = -(P->lambda_im[0] * T[0] + P->lambda_im[1] * T[1]);",
     "double ei = -(P->lambda_im[1] * T[0] + P->lambda_im[0] * T[1]);",
     ["test_equal_kappa_unequal_lambda_two_sided_closed_form"], KPINS),
    ("kappa_step_scale", "double s = sqrt(ki * dt);", "double s = sqrt(dt);",
     ["test_equal_kappa_is_the_constant_coefficient_walk"], KPINS),
    ("kappa_exit_share", "T[si] += fr * dt;", "T[si] += dt;", ["test_occupation_shares_sum_to_the_step"], KPINS),
    # the split of an interface step's time between the sides (ways that keep
    # the sum and converge to the same continuum limit)
    ("kappa_split_all_to_start", KAPPA_SPLIT,
     KAPPA_SPLIT.replace("T[si] += dt - 0.5 * (dt - tg) * pi_;\n            T[sj] += 0.5 * (dt - tg) * pi_;",
                         "T[si] += dt;").replace(
         "T[si] += tg + 0.5 * (dt - tg) * pj;\n            T[sj] += 0.5 * (dt - tg) * (2.0 - pj);", "T[si] += dt;"),
     ["test_interface_split_matches_the_exact_scheme"], KPINS),
    ("kappa_split_all_to_resume", KAPPA_SPLIT,
     KAPPA_SPLIT.replace("T[si] += dt - 0.5 * (dt - tg) * pi_;\n            T[sj] += 0.5 * (dt - tg) * pi_;",
                         "T[si] += dt;").replace(
         "T[si] += tg + 0.5 * (dt - tg) * pj;\n            T[sj] += 0.5 * (dt - tg) * (2.0 - pj);", "T[sj] += dt;"),
     ["test_interface_split_matches_the_exact_scheme"], KPINS),
    ("kappa_split_p_swapped",
     "T[si] += dt - 0.5 * (dt - tg) * pi_;\n            T[sj] += 0.5 * (dt - tg) * pi_;",
     "T[si] += dt - 0.5 * (dt - tg) * pj;\n            T[sj] += 0.5 * (dt - tg) * pj;",
     ["test_interface_split_matches_the_exact_scheme"], KPINS),
    ("kappa_split_tg_to_other",
     "T[si] += tg + 0.5 * (dt - tg) * pj;\n            T[sj] += 0.5 * (dt - tg) * (2.0 - pj);",
     "T[sj] += tg + 0.5 * (dt - tg) * (2.0 - pj);\n            T[si] += 0.5 * (dt - tg) * pj;",
     ["test_interface_split_matches_the_exact_scheme"], KPINS),
]


@pytest.mark.parametrize("name,orig,mut,pins,pin_file", [m if len(m) == 5 else (*m, PINS) for m in MUTANTS],
                         ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, orig, mut, pins, pin_file, tmp_path):
    src = open(SRC).read()
    # the TE walk precedes the discontinuous-kappa section; each mutant edits its own section
    cut = src.index(KAPPA_SECTION)
    head, tail = src[:cut], src[cut:]
    if pin_file == KPINS:
        assert tail.count(orig) == 1, name
        tail = tail.replace(orig, mut)
    else:
        assert head.count(orig) == 1, name
        head = head.replace(orig, mut)
    msrc = tmp_path / "mut.c"
    msrc.write_text(head + tail)
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                           str(msrc), "-o", str(lib), "-lm", "-lpthread"])
    env = dict(os.environ, SDD_ORACLE_LIB=str(lib))
    sel = " or ".join(pins)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, pin_file), "-k", sel],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.stdout[-2000:])
