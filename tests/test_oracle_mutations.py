"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
the pins in ``test_oracle_pins.py`` catch every one of them.

Each mutation edits one expression of ``oracle/oreg_oracle.c``, builds the
copy with gcc into a temporary directory and runs the pin suite against it in
a subprocess (``OREG_ORACLE_LIB`` selects the build).  A mutation that
survives would mean the pins cannot tell that slip from the paper's method.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oreg_oracle.c")

MUTATIONS = {
    "peculiar_velocity_sign": ("C[a] = (double)CVEL[i][a] - u[a];",
                               "C[a] = (double)CVEL[i][a] + u[a];"),
    # either trace term alone is redundant (each tensor is trace-free); drop both
    "drop_both_trace_terms": ("(a == b ? C2 / D : 0.0)) * S[a][b];|(a == b ? ck2 / D : 0.0);",
                              "0.0) * S[a][b];|0.0;"),
    "prefactor_theta_power": ("fo[i] = feq[i] / (2.0 * rho * theta * theta) * acc;",
                              "fo[i] = feq[i] / (2.0 * rho * theta) * acc;"),
    "prefactor_missing_rho": ("fo[i] = feq[i] / (2.0 * rho * theta * theta) * acc;",
                              "fo[i] = feq[i] / (2.0 * theta * theta) * acc;"),
    "guided_cu_sign": ("prod *= pref * (c2 - 1.0 + c * u[a] + u[a] * u[a] + theta);",
                       "prod *= pref * (c2 - 1.0 - c * u[a] + u[a] * u[a] + theta);"),
    "guided_drop_u2": ("prod *= pref * (c2 - 1.0 + c * u[a] + u[a] * u[a] + theta);",
                       "prod *= pref * (c2 - 1.0 + c * u[a] + theta);"),
    "poly2_as_printed": ("cu * cu / (2.0 * theta0 * theta0) - uu / (2.0 * theta0));",
                         "cu * cu / (2.0 * theta0 * theta0));"),
    "relaxation_factor": ("fpost[i] = feq[i] + (1.0 - 1.0 / tau) * fo[i];",
                          "fpost[i] = feq[i] + (1.0 / tau) * fo[i];"),
    "streaming_direction": ("const int xd = wrap(x + CVEL[i][0], nx);",
                            "const int xd = wrap(x - CVEL[i][0], nx);"),
    "stress_index": ("const double t = (double)(CVEL[k][a] * CVEL[k][b]) - (a == b ? ck2 / D : 0.0);",
                     "const double t = (double)(CVEL[k][a] * CVEL[k][a]) - (a == b ? ck2 / D : 0.0);"),
    "stress_from_f_not_fneq": ("for (int k = 0; k < Q; ++k) fneq[k] = f[k] - feq[k];",
                               "for (int k = 0; k < Q; ++k) fneq[k] = f[k];"),
    "velocity_component_swap": ("*ux = jx / r;", "*ux = jy / r;"),
    "bounceback_half_reverse": ("if (CVEL[j][0] == -CVEL[i][0] && CVEL[j][1] == -CVEL[i][1]) return j;",
                                "if (CVEL[j][0] == -CVEL[i][0] && CVEL[j][1] == CVEL[i][1]) return j;"),
    "bgk_rate": ("fpost[i] = f[i] - (f[i] - feq[i]) / tau;", "fpost[i] = f[i] - (f[i] - feq[i]) * tau;"),
    "energy_pressure": ("etot += 0.5 * (D * rho * theta + rho * (ux * ux + uy * uy));",
                        "etot += 0.5 * (rho * theta + rho * (ux * ux + uy * uy));"),
    "diagonal_velocity": ("{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};",
                          "{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    olds, news = MUTATIONS[name]
    src = open(SRC).read()
    for old, new in zip(olds.split("|"), news.split("|")):
        assert src.count(old) == 1, f"mutation anchor not unique/absent: {name}"
        src = src.replace(old, new)
    mutated = tmp_path / "oreg_oracle.c"
    mutated.write_text(src)
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(mutated), "-lm"],
                   check=True)
    env = dict(os.environ, OREG_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
