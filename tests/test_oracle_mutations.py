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


# mistakes in the general operator (closed links, diagonal term, excluded
# cells), caught by tests/test_oracle_general.py
MUTATIONS_GEN = {
    "gen-sigma-sign": ("y[c] -= sigma[c] * x[c];", "y[c] += sigma[c] * x[c];"),
    "gen-never-singular": ("    int singular = 1;\n", "    int singular = 0;\n"),
    "gen-diag-without-sigma": ("dg[c] = s * ih2 + (sigma ? sigma[c] : 0.0);", "dg[c] = s * ih2;"),
    "gen-mean-over-all-cells": ("    double bmean = (singular && nact) ? bsum / (double)nact : 0.0;",
                                "    double bmean = (singular && nact) ? bsum / (double)N : 0.0;"),
}

PY_MUTATIONS_GEN = {
    "gen-project-keeps-closed-links": ("    return tuple(np.where(o[m], u[m], 0.0) for m in range(3))\n",
                                       "    return tuple(u)\n"),
}


def _run_pins(pin_file, env):
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--timeout",
                           "60", os.path.join(ROOT, "tests", pin_file)],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("name", sorted(MUTATIONS_GEN))
def test_general_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS_GEN[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutated = tmp_path / "pp_oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libpp_oracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                           str(mutated), "-lm"])
    env = dict(os.environ, PP_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = _run_pins("test_oracle_general.py", env)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(PY_MUTATIONS_GEN))
def test_general_pins_catch_python_mutation(name, tmp_path):
    """The same for the oracle's Python layer: a mutated copy of the package
    is put first on the path."""
    import shutil
    old, new = PY_MUTATIONS_GEN[name]
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    init = pkg / "__init__.py"
    src = init.read_text()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    init.write_text(src.replace(old, new))
    env = dict(os.environ, PYTHONPATH=str(tmp_path) + os.pathsep + os.environ.get("PYTHONPATH", ""),
               PP_ORACLE_LIB=os.path.join(ROOT, "oracle", "libpp_oracle.so"), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c",
                        "import sys, pytest; import oracle; assert oracle.__file__.startswith(sys.argv[1]);"
                        "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', sys.argv[2]]))",
                        str(tmp_path), os.path.join(ROOT, "tests", "test_oracle_general.py")],
                       cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}{r.stderr[-2000:]}"


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
