"""Planted mistakes: each variant of the oracle source carries one plausible bug (a dropped
term, a wrong sign, a wrong index or factor), is compiled on the CPU, and the pins named next
to it are run against it in a subprocess.  Every variant must make at least one pin fail,
which shows that the pins constrain the oracle rather than only restate it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mpr_oracle.c")

P = "tests/test_oracle_primitives.py::"
M = "tests/test_oracle_method.py::"

MUTANTS = {
    "philox_multiplier": ("(uint64_t)0xD2511F53u * x0", "(uint64_t)0xD2511F55u * x0",
                          [P + "test_philox_known_answers"]),
    "philox_key_bump": ("k1 += 0xBB67AE85u;", "k1 += 0xBB67AE87u;",
                        [P + "test_philox_known_answers"]),
    "field_drops_a_neighbour": ("for (int k = 0; k < n; ++k) { c += cos",
                                "for (int k = 0; k < n - 1; ++k) { c += cos",
                                [P + "test_local_field_and_site_energy_by_hand",
                                 M + "test_single_free_spin_matches_quadrature"]),
    "energy_sign_in_delta": ("double dE = orc_site_energy(H, W, phi, boundary, q, J, y, x, phi_p)\n"
                             "              - orc_site_energy(H, W, phi, boundary, q, J, y, x, phi[i]);",
                             "double dE = orc_site_energy(H, W, phi, boundary, q, J, y, x, phi[i])\n"
                             "              - orc_site_energy(H, W, phi, boundary, q, J, y, x, phi_p);",
                             [M + "test_single_free_spin_matches_quadrature"]),
    "metropolis_exponent_sign": ("exp(-dE / T)", "exp(dE / T)",
                                 [M + "test_single_free_spin_matches_quadrature"]),
    "overrelax_factor": ("2.0 * psi / q - phi_i", "psi / q - phi_i",
                         [P + "test_overrelax_closed_form_equal_neighbours",
                          P + "test_overrelax_conserves_energy_and_is_involution"]),
    "overrelax_atan2_operands": ("atan2(S, C)", "atan2(C, S)",
                                 [P + "test_overrelax_closed_form_equal_neighbours"]),
    "row_index_uses_height": ("if (y > 0) nb[n++] = (y - 1) * W + x;",
                              "if (y > 0) nb[n++] = (y - 1) * H + x;",
                              [P + "test_local_field_and_site_energy_by_hand"]),
    "bond_energy_drops_q": ("if (!mask || (mask[i] && mask[j])) { s += cos(q * (phi[i] - phi[j])); ++c; }\n"
                            "            }\n            /* lower",
                            "if (!mask || (mask[i] && mask[j])) { s += cos(phi[i] - phi[j]); ++c; }\n"
                            "            }\n            /* lower",
                            [P + "test_staggered_configuration_energy",
                             P + "test_twisted_periodic_energy_closed_form"]),
    "periodic_wrap_wrong_site": ("if (xr == W) xr = (boundary == ORC_PERIODIC) ? 0 : -1;",
                                 "if (xr == W) xr = (boundary == ORC_PERIODIC) ? 1 : -1;",
                                 [P + "test_twisted_periodic_energy_closed_form"]),
    "map_divides_by_max": ("TWO_PI * ((z[i] - lo) / (hi - lo))", "TWO_PI * ((z[i] - lo) / hi)",
                           [P + "test_map_endpoints_and_equivariance"]),
    "proposal_range_unchecked": ("if (phi_p < 0.0 || phi_p > TWO_PI) return dec | ORC_DEC_OUTSIDE;",
                                 "if (phi_p < -1e300) return dec | ORC_DEC_OUTSIDE;",
                                 [M + "test_single_free_spin_matches_quadrature"]),
    "temperature_ratio_inverted": ("double r = den <= 1e-300 ? 2.0 : num / den;",
                                   "double r = den <= 1e-300 ? 2.0 : den / num;",
                                   [M + "test_temperature_recovery"]),
    "window_control_inverted": ("a = clampd(a * A / g->acc_target, 1e-3, 1.0);",
                                "a = clampd(a * g->acc_target / (A + 1e-12), 1e-3, 1.0);",
                                [M + "test_window_control_reaches_target_acceptance"]),
    "average_overwrites": ("if (!c->mask[i]) a[i] += p[i];", "if (!c->mask[i]) a[i] = p[i];",
                           [M + "test_ramp_is_reproduced_at_low_temperature"]),
    "pair_member_words_swapped": ("if ((kx & 1) == 0) { *wa = out[0]; *wb = out[1]; }",
                                  "if ((kx & 1) == 1) { *wa = out[0]; *wb = out[1]; }",
                                  [P + "test_site_words_pairing_and_uniqueness"]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new, tests = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found exactly once: %s" % name
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-shared",
                           "-fPIC", "-I", os.path.join(ROOT, "oracle"), "-o", str(so), str(mut),
                           "-lm"])
    env = dict(os.environ, MPR_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-p", "no:randomly"] + tests, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutant %s:\n%s" % (name, r.stdout[-2000:])

