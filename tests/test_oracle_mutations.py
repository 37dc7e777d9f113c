"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch every one of them: a dropped term, a flipped sign, a wrong index, a
transposed operand, a missing wall or mean treatment."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pp_oracle.c")

MUTATIONS = {
    "flux-sign": ("s += beta_high(g, beta, ijk, m) * (x[up] - x[c]);",
                  "s += beta_high(g, beta, ijk, m) * (x[c] - x[up]);"),
    "flux-face-index": ("s += beta_high(g, beta, ijk, m) * (x[up] - x[c]);",
                        "s += beta_low(g, beta, ijk, m) * (x[up] - x[c]);"),
    "div-dropped-term": ("s += (hi - lo) / h;", "s += hi / h;"),
    "project-sign": ("u[m][c] = us[m][c] - dt * beta[m][c] * grad;",
                     "u[m][c] = us[m][c] + dt * beta[m][c] * grad;"),
    "face-average": ("2.0 / (rho[lo] + rho[c])", "0.5 * (1.0 / rho[lo] + 1.0 / rho[c])"),
    "sor-link-swap": ("A[2 * m] = beta_low(g, beta, ijk, m) * ih2;",
                      "A[2 * m] = beta_high(g, beta, ijk, m) * ih2;"),
    "adjoint-sign": ("gb[m][c] = (grhs[c] - grhs[dn]) * (p[c] - p[dn]) / (h * h);",
                     "gb[m][c] = (grhs[dn] - grhs[c]) * (p[c] - p[dn]) / (h * h);"),
    "no-mean-removal": ("    memcpy(b, rhs, sizeof(double) * N);\n    remove_mean(b, N);",
                        "    memcpy(b, rhs, sizeof(double) * N);"),
    "wall-as-periodic": ("        if (g->bc[m] == 1)\n            return -1;\n", ""),
    "transposed-coords": ("ijk[0] = c % g->n[0];", "ijk[0] = c % g->n[1];"),
    "sor-omega-ignored": ("p[c] = (1.0 - omega) * p[c] + (omega / A7) * (sum - A8);",
                          "p[c] = (sum - A8) / A7;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutated = tmp_path / "pp_oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libpp_oracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                           str(mutated), "-lm"])
    env = dict(os.environ, PP_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--timeout", "60",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
