"""The oracle's pins must catch plausible mistakes.  Each case plants one mistake in a copy of
the oracle's C source (on the CPU), builds it, and runs the pin suite against that build; the
suite has to fail.  The shipped oracle is never modified."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nbody_oracle.c")

MUTATIONS = {
    "jerk_sign": ("jx += mj * (ux * inv_r3 - 3.0 * du * dx * inv_r5);",
                  "jx += mj * (ux * inv_r3 + 3.0 * du * dx * inv_r5);"),
    "repulsive": ("const double dx = x[3 * j + 0] - x[3 * i + 0];",
                  "const double dx = x[3 * i + 0] - x[3 * j + 0];"),
    "pot_power": ("p -= mj * inv_r;", "p -= mj * inv_r3;"),
    "self_term": ("if (j == i) continue;\n            const double dx = x[3 * j + 0] - x[3 * i + 0];\n            const double dy = x[3 * j + 1] - x[3 * i + 1];\n            const double dz = x[3 * j + 2] - x[3 * i + 2];\n            const double ux",
                  "const double dx = x[3 * j + 0] - x[3 * i + 0];\n            const double dy = x[3 * j + 1] - x[3 * i + 1];\n            const double dz = x[3 * j + 2] - x[3 * i + 2];\n            const double ux"),
    "predictor_jerk": ("k[c] * D * D * D / 6.0", "k[c] * D * D * D / 2.0"),
    "corrector_swap": ("(4.0 * k0[c] + 2.0 * k1[c]) / dt", "(2.0 * k0[c] + 4.0 * k1[c]) / dt"),
    "corrector_a3": ("a3[c] * dt * dt * dt * dt * dt / 120.0", "a3[c] * dt * dt * dt * dt * dt / 24.0"),
    "crit_no_a3dt": ("a2p[c] = a2[c] + a3[c] * dt;", "a2p[c] = a2[c];"),
    "crit_no_sqrt": ("return sqrt(nu * crit_num / crit_den);", "return nu * crit_num / crit_den;"),
    "no_commensurability": ("if (t % two_dt == 0) return l - 1;", "return l - 1;"),
    "energy_double_count": ("*epot = (double)(-0.5L * w);", "*epot = (double)(-w);"),
    "initial_dt_inverted": ("return nu * na / nk;", "return nu * nk / na;"),
    "scale_jerk_factor": ("k += m[j] * (speed * inv_r3 + 3.0 * du * dist * inv_r3 / s);",
                          "k += m[j] * (speed * inv_r3 + du * dist * inv_r3 / s);"),
    "scale_no_mass": ("a += m[j] * dist * inv_r3;", "a += dist * inv_r3;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = ob.build(src=str(mutated), lib=str(tmp_path / "mutant.so"))
    env = dict(os.environ, NBODY_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
