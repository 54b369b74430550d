"""The pins constrain the oracle: each test here plants one plausible mistake in a
copy of the oracle's C source (on the CPU), builds it, and checks that the pin
meant to catch it fails -- while the same pin passes on the unmodified source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
ORACLE = os.path.join(ROOT, "oracle")

# (name, file, original text, planted mistake, pin that must fail)
MUTANTS = [
    ("half_coupling", "xy_oracle.c", "((2.0 * beta) * ai) * aj", "((1.0 * beta) * ai) * aj",
     "test_oracle_physics.test_l2_exact_averages(1.12)"),
    ("inverted_rule", "xy_oracle.c", "return e < one_minus_u;", "return e > one_minus_u;",
     "test_oracle_physics.test_l2_exact_averages(0.5)"),
    ("unsigned_projection", "xy_oracle.c", "double xb = ((2.0 * beta) * ai) * aj;",
     "double xb = ((2.0 * beta) * fabs(ai)) * fabs(aj);",
     "test_oracle_physics.test_beta_infinite_clusters_are_same_sign_domains()"),
    ("reflection_sign", "xy_oracle.c", "c[i] = store(c[i] - g * r[0], storage32);",
     "c[i] = store(c[i] + g * r[0], storage32);",
     "test_oracle_physics.test_reflection_geometry_and_cluster_coherence()"),
    ("coin_by_site", "xy_oracle.c", "if (!orc_coin(seed, rep, t, label[i])) continue;",
     "if (!orc_coin(seed, rep, t, i)) continue;",
     "test_oracle_physics.test_reflection_geometry_and_cluster_coherence()"),
    ("bfs_left_link", "xy_oracle.c", "int on[4] = {bx[k], by[k], bx[nb[2]], by[nb[3]]};",
     "int on[4] = {bx[k], by[k], bx[k], by[nb[3]]};",
     "test_oracle_ccl.test_l2_every_link_subset()"),
    ("energy_drops_y", "xy_oracle.c", "obs[0] = -(scx + scy) / n;", "obs[0] = -(scx) / n;",
     "test_oracle_physics.test_l2_exact_averages(0.5)"),
    ("m2_normalisation", "xy_oracle.c", "obs[1] = (sc * sc + ss * ss) / (n * n);",
     "obs[1] = (sc * sc + ss * ss) / n;", "test_oracle_physics.test_l2_exact_averages(0.5)"),
    ("sin_sign", "xy_oracle.c", "ssx += s[i] * c[j] - c[i] * s[j];", "ssx += s[i] * c[j] + c[i] * s[j];",
     "test_oracle_physics.test_measure_matches_angle_formulas()"),
    ("pcc_direction", "xy_oracle.c", "*beta += (bu < target) ? db : -db;", "*beta += (bu < target) ? -db : db;",
     "test_oracle_physics.test_pcc_direction_of_steps()"),
    ("down_neighbour", "xy_oracle.c", "static int64_t down_of(int64_t i, int64_t L) { return ((i / L + 1) % L) * L + i % L; }",
     "static int64_t down_of(int64_t i, int64_t L) { return ((i / L + 1) % L) * L + (i + 1) % L; }",
     "test_oracle_physics.test_measure_matches_angle_formulas()"),
    ("fourier_along_y", "xy_oracle.c", "double kx = 2.0 * pi * (double)(i % L) / (double)L;",
     "double kx = 2.0 * pi * (double)(i / L) / (double)L;",
     "test_oracle_physics.test_fourier_magnetisation_closed_forms()"),
    ("fourier_drops_sin_part", "xy_oracle.c", "obs[7] = (cre * cre + cim * cim + sre * sre + sim * sim) / (n * n);",
     "obs[7] = (cre * cre + sre * sre) / (n * n);",
     "test_oracle_physics.test_measure_matches_angle_formulas()"),
    ("wrap_ignores_y", "xy_oracle.c", "if (uy[j] != ey) *wrap |= 2;", "if (uy[j] != ey) *wrap |= 0;",
     "test_oracle_wrap.test_hand_built_sets()"),
    ("wrap_left_step", "xy_oracle.c", "int64_t dx[4] = {1, 0, -1, 0}, dy[4] = {0, 1, 0, -1};",
     "int64_t dx[4] = {1, 0, 1, 0}, dy[4] = {0, 1, 0, -1};", "test_oracle_wrap.test_l2_every_link_subset_against_the_cover()"),
    ("wrap_x_as_y", "xy_oracle.c", "if (ux[j] != ex) *wrap |= 1;", "if (ux[j] != ex) *wrap |= 2;",
     "test_oracle_wrap.test_symmetries()"),
    ("perc_rule_direction", "xy_oracle.c", "*beta += (p < target) ? db : -db;", "*beta += (p > target) ? db : -db;",
     "test_oracle_wrap.test_percolation_pcc_direction_of_steps()"),
    ("philox_key_bump", "xy_oracle.c", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;",
     "test_oracle_philox.test_philox4x32_known_answers([0, 0, 0, 0], [0, 0], "
     "[0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8])"),
]


def _build(tmp, name, fname, old, new):
    d = tmp / name
    d.mkdir()
    for src in ("xy_oracle.c", "metropolis.c"):
        text = open(os.path.join(ORACLE, src)).read()
        if src == fname:
            assert text.count(old) == 1, (name, old)
            text = text.replace(old, new)
        (d / src).write_text(text)
    lib = d / "lib.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib),
                    str(d / "xy_oracle.c"), str(d / "metropolis.c"), "-lm"], check=True)
    return str(lib)


def _pin_passes(lib, call):
    mod = call.split(".")[0]
    code = ("import sys; sys.path[:0] = [%r, %r]; import %s; %s" % (ROOT, TESTS, mod, call))
    env = dict(os.environ, XY_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    return r.returncode == 0


@pytest.mark.parametrize("name,fname,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(tmp_path, name, fname, old, new, pin):
    good = _build(tmp_path, "good", fname, old, old)
    assert _pin_passes(good, pin), "pin fails on the unmodified oracle"
    bad = _build(tmp_path, "bad", fname, old, new)
    assert not _pin_passes(bad, pin), "pin did not catch %s" % name
