"""Plant plausible mistakes in copies of the D3Q27 oracle (on the CPU) and
check that the pins in ``test_oracle3_pins.py`` catch every one of them.

Each mutation edits ``oracle/oreg_oracle3.c``, builds the copy with gcc into
a temporary directory and runs the 3D pin suite against it in a subprocess
(``OREG_ORACLE3_LIB`` selects the build).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oreg_oracle3.c")

MUTATIONS = {
    # the printed D2Q9 axis factor, whose three-axis product flips the sign
    "printed_2d_axis_sign": ("const double pref = (2.0 * c2 - 1.0) / pow(2.0, c2);",
                             "const double pref = (1.0 - 2.0 * c2) / pow(2.0, c2);"),
    "trace_with_d2": ("(a == b ? C2 / D : 0.0)) * S[a][b];|(a == b ? ck2 / D : 0.0);",
                      "(a == b ? C2 / 2.0 : 0.0)) * S[a][b];|(a == b ? ck2 / 2.0 : 0.0);"),
    "stress_trace_only": ("(a == b ? ck2 / D : 0.0);", "(a == b ? ck2 / 2.0 : 0.0);"),
    "prefactor_theta_power": ("fo[i] = feq[i] / (2.0 * rho * theta * theta) * acc;",
                              "fo[i] = feq[i] / (2.0 * rho * theta) * acc;"),
    "peculiar_velocity_sign": ("C[a] = (double)CV[i][a] - u[a];", "C[a] = (double)CV[i][a] + u[a];"),
    "streaming_direction_z": ("const int zd = wrap(z + CV[i][2], nz);",
                              "const int zd = wrap(z - CV[i][2], nz);"),
    "velocity_table_z": ("CV[i][2] = i / 9 - 1;", "CV[i][2] = (i / 3) % 3 - 1;"),
    "relaxation_factor": ("fpost[i] = feq[i] + (1.0 - 1.0 / tau) * fo[i];",
                          "fpost[i] = feq[i] + (1.0 / tau) * fo[i];"),
    "poly2_as_printed": ("cu * cu / (2.0 * theta0 * theta0) - uu / (2.0 * theta0));",
                         "cu * cu / (2.0 * theta0 * theta0));"),
    "guided_drop_u2": ("prod *= pref * (c2 - 1.0 + c * u[a] + u[a] * u[a] + theta);",
                       "prod *= pref * (c2 - 1.0 + c * u[a] + theta);"),
    "momentum_axis": ("for (int a = 0; a < D; ++a) j[a] += (double)CV[i][a] * f[i];",
                      "for (int a = 0; a < D; ++a) j[a] += (double)CV[i][(a + 1) % D] * f[i];"),
    "stress_index": ("const double t = (double)(CV[k][a] * CV[k][b]) - (a == b ? ck2 / D : 0.0);",
                     "const double t = (double)(CV[k][a] * CV[k][a]) - (a == b ? ck2 / D : 0.0);"),
    "stress_from_f_not_fneq": ("for (int k = 0; k < Q; ++k) fneq[k] = f[k] - feq[k];",
                               "for (int k = 0; k < Q; ++k) fneq[k] = f[k];"),
    "bgk_rate": ("fpost[i] = f[i] - (f[i] - feq[i]) / tau;", "fpost[i] = f[i] - (f[i] - feq[i]) * tau;"),
    "energy_pressure": ("etot += 0.5 * (D * rho * theta + rho * uu);",
                        "etot += 0.5 * (2.0 * rho * theta + rho * uu);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    olds, news = MUTATIONS[name]
    src = open(SRC).read()
    for old, new in zip(olds.split("|"), news.split("|")):
        assert src.count(old) == 1, f"mutation anchor not unique/absent: {name}"
        src = src.replace(old, new)
    mutated = tmp_path / "oreg_oracle3.c"
    mutated.write_text(src)
    lib = tmp_path / "libmut3.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(mutated), "-lm"],
                   check=True)
    env = dict(os.environ, OREG_ORACLE3_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle3_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
