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

# (name, original text, mutated text, pins expected to fail)
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
    ("table_index_shift", "out[0] = (1.0 - lam) * gw[2 * i] + lam * gw[2 * i + 2];",
     "out[0] = (1.0 - lam) * gw[2 * i + 2] + lam * gw[2 * i + 4];", ["test_table_interpolation_linear_exact"]),
    ("air_phase", "if (P->freq_hz > 0.0) {", "if (sigma == 0.0) return P->alpha_direct;\n    if (P->freq_hz > 0.0) {",
     ["test_layered_halfspace_is_1d"]),
    ("region_order", "for (int r = 0; r < P->n_regions; ++r)\n        if (in_primitive",
     "for (int r = P->n_regions - 1; r >= 0; --r)\n        if (in_primitive", ["test_region_predicate"]),
]


@pytest.mark.parametrize("name,orig,mut,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, orig, mut, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) == 1, name
    msrc = tmp_path / "mut.c"
    msrc.write_text(src.replace(orig, mut))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                           str(msrc), "-o", str(lib), "-lm", "-lpthread"])
    env = dict(os.environ, SDD_ORACLE_LIB=str(lib))
    sel = " or ".join(pins)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py"), "-k", sel],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, (name, r.stdout[-2000:])
