"""The oracle's pins catch plausible mistakes (CPU only).

Each case below plants one mistake in a copy of the oracle's C sources -- a
wrong sign, a dropped term, a transposed operand, a mistyped coefficient, a
relaxed comparison -- builds the copy, and runs the pin tests of that part of
the oracle against it (through ORACLE_LIB).  The pins must fail for every
mutant, and pass for an unchanged copy built the same way.  The mistakes are
planted here, on the CPU, never in the code under test.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
ORACLE = os.path.join(REPO, "oracle")

PINS = "tests/test_oracle_pins.py"

# name: (file, original text, planted mistake, pin test files)
MUTANTS = {
    "equilibrium-pressure-term-sign": (
        "rhs_body.h", "SC ln_Kc = -dG + (double)m->sum_nu[j] * ln_patm_RT;",
        "SC ln_Kc = -dG - (double)m->sum_nu[j] * ln_patm_RT;", [PINS]),
    "third-body-efficiencies-dropped": (
        "rhs_body.h", "mj += m->alpha[(size_t)j * N + k] * C[k];", "mj += C[k];", [PINS]),
    "energy-equation-sign": (
        "rhs_body.h", "f[0] = -heat / cp_mass;", "f[0] = heat / cp_mass;", [PINS]),
    "third-product-slot-dropped": (
        "rhs_body.h", "for (int s = 0; s < 3; ++s) if (ps[s] >= 0) omega[ps[s]] += q;",
        "for (int s = 0; s < 2; ++s) if (ps[s] >= 0) omega[ps[s]] += q;", [PINS]),
    "rodas-coefficient-typo": (
        "rodas.c", "A43 = 0.9986419139977817", "A43 = 0.9886419139977817", [PINS]),
    "lu-smallest-pivot": (
        "rodas.c", "if (v > amax) { amax = v; p = i; }", "if (v < amax) { amax = v; p = i; }",
        [PINS]),
    "lu-transposed-operand": (
        "rodas.c", "A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];",
        "A[(size_t)i * n + j] -= l * A[(size_t)j * n + k];", [PINS]),
    "mapping-threshold-not-strict": (
        "mapping.c", "if (!(Z[i] < Z_tol)) continue;", "if (!(Z[i] <= Z_tol)) continue;",
        ["tests/test_oracle_mapping.py"]),
    "gelu-wrong-scale": (
        "mlp.c", "static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }",
        "static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / 2.0)); }",
        ["tests/test_oracle_surrogate.py"]),
    "troe-asymmetry-sign": (
        "rhs_body.h", "const SC f1 = x / (nn - 0.14 * x);", "const SC f1 = x / (nn + 0.14 * x);",
        ["tests/test_oracle_falloff.py"]),
    "troe-width-constant": (
        "rhs_body.h", "nn = 0.75 - 1.27 * lFc;", "nn = 0.75 - 1.72 * lFc;",
        ["tests/test_oracle_falloff.py"]),
    "troe-centre-constant": (
        "rhs_body.h", "const SC c = -0.4 - 0.67 * lFc", "const SC c = -0.4 - 0.76 * lFc",
        ["tests/test_oracle_falloff.py"]),
    "enthalpy-polynomial-term": (
        "chem.c", "+ a[4] * T * T * T * T / 5.0 + a[5] / T;", "+ a[4] * T * T * T * T / 4.0 + a[5] / T;",
        [PINS]),
    "entropy-log-term": (
        "chem.c", "s_R[k] = a[0] * lnT + a[1] * T", "s_R[k] = a[0] * T + a[1] * T", [PINS]),
    "jacobian-heat-capacity-derivative": (
        "chem.c", "return a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T * T + 4.0 * a[4] * T * T * T;",
        "return a[1] + 2.0 * a[2] * T + 2.0 * a[3] * T * T + 4.0 * a[4] * T * T * T;", [PINS]),
    "error-norm-scale-ignores-new-state": (
        "rodas.c", "double sc = o->atol + o->rtol * fmax(fabs(y[i]), fabs(ynew[i]));",
        "double sc = o->atol + o->rtol * fabs(y[i]);", [PINS]),
    "controller-safety-factor": (
        "rodas.c", "fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.25)))", "fmin(5.0, fmax(0.2, 0.8 * pow(e, -0.25)))",
        [PINS]),
    "controller-growth-bound": (
        "rodas.c", "fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.25)))", "fmin(4.0, fmax(0.2, 0.9 * pow(e, -0.25)))",
        [PINS]),
    "controller-exponent": (
        "rodas.c", "fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.25)))", "fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.2)))",
        [PINS]),
    "gelu-derivative": (
        "mlp.c", "z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI)", "z * exp(-z * z) / sqrt(2.0 * M_PI)",
        ["tests/test_oracle_surrogate.py"]),
    "gate-residual-sign": (
        "mlp.c", "if (!(fabs(*T + dT - Th) <= tau_T)) return 0;",
        "if (!(fabs(*T - dT - Th) <= tau_T)) return 0;", ["tests/test_oracle_surrogate.py"]),
    "plog-interpolation-end-swapped": (
        "rhs_body.h",
        "const double w = (log(p) - log(t[4 * i])) / (log(t[4 * i + 4]) - log(t[4 * i]));",
        "const double w = (log(t[4 * i + 4]) - log(p)) / (log(t[4 * i + 4]) - log(t[4 * i]));",
        ["tests/test_oracle_plog.py"]),
}


def _build(src_dir, out):
    from oracle.build import SOURCES
    cmd = ["gcc", "-std=gnu11", "-O1", "-march=x86-64-v3", "-ffp-contract=off", "-fno-math-errno",
           "-fopenmp", "-fPIC", "-shared", "-w", "-o", out] + \
          [os.path.join(src_dir, s) for s in SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=True)


def _copy(dst):
    os.makedirs(dst)
    for f in os.listdir(ORACLE):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(ORACLE, f), dst)


def _pins(lib, files):
    env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                           "-p", "no:cacheprovider"] + files,
                          cwd=REPO, env=env, capture_output=True, text=True, timeout=900)


def _one(tmp, name):
    fname, old, new, files = MUTANTS[name]
    d = os.path.join(tmp, name)
    _copy(d)
    path = os.path.join(d, fname)
    txt = open(path).read()
    assert txt.count(old) == 1, (name, txt.count(old))
    open(path, "w").write(txt.replace(old, new))
    lib = os.path.join(d, "liboracle.so")
    _build(d, lib)
    return _pins(lib, files)


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("mutants"))
    ctrl = os.path.join(tmp, "control")
    _copy(ctrl)
    _build(ctrl, os.path.join(ctrl, "liboracle.so"))
    files = sorted({f for m in MUTANTS.values() for f in m[3]})
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        fut_ctrl = ex.submit(_pins, os.path.join(ctrl, "liboracle.so"), files)
        futs = {name: ex.submit(_one, tmp, name) for name in MUTANTS}
        return fut_ctrl.result(), {name: f.result() for name, f in futs.items()}


def test_unchanged_copy_passes_the_pins(outcomes):
    ctrl, _ = outcomes
    assert ctrl.returncode == 0, ctrl.stdout[-3000:] + ctrl.stderr[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_the_planted_mistake(outcomes, name):
    _, res = outcomes
    r = res[name]
    # exit status 1: tests ran and at least one failed (not a crash or a usage error)
    assert r.returncode == 1 and " failed" in r.stdout, \
        f"mutant {name} survived (status {r.returncode}):\n{r.stdout[-2000:]}{r.stderr[-1000:]}"
