"""Pin audit: plausible mistakes planted in the oracle must fail its pins.

Each mutant is the oracle's C source with one plausible slip (a wrong sign or
tie rule, a dropped term, a wrong index, a wrong truncation) or a Python-level
slip in the normalisation, built into a temporary library and run against the
pin tests in a child process.  A mutant that survives would mean the pins do
not constrain that part of the oracle.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hs_oracle.c")
PINS = ["tests/test_oracle_pipeline.py", "tests/test_oracle_golden.py", "tests/test_oracle_stats.py",
        "tests/test_oracle_bruteforce.py", "tests/test_oracle_physics.py", "tests/test_oracle_invariants.py",
        "tests/test_oracle_presto.py", "tests/test_oracle_candidates.py", "tests/test_oracle_table.py"]

C_MUTANTS = {
    "greedy-tie-moves": ("if (b > a) { d += 1; v = b; }", "if (b >= a) { d += 1; v = b; }"),
    "wrong-neighbour": ("k * n + d + 1);", "k * n + d + 2);"),
    "dropped-term": ("S = S + v;", "S = v;"),
    "snr-tie-to-larger-k": ("snr > best)", "snr >= best)"),
    "no-mean": ("fmaf(S, rs[k - 1], nm[k - 1])", "fmaf(S, rs[k - 1], 0.0f)"),
    "truncation-off-by-one": ("int64_t k = (len - 1) / reach;", "int64_t k = (len - 2) / reach;"),
    "no-drift-in-sum": ("{ d += 1; v = b; } else { v = a; }", "{ d += 1; v = a; } else { v = a; }"),
    "2d-row-not-scaled": ("int64_t row = k * z - z_min;", "int64_t row = z - z_min;"),
    "drift-before-step": ("kb = (int32_t)k; db = (int32_t)d;", "kb = (int32_t)k; db = (int32_t)(d > 0 ? d - 1 : 0);"),
    "presto-round-down": ("return (2 * h * n + K) / (2 * K);", "return (2 * h * n) / (2 * K);"),
    "presto-half-down": ("return (2 * h * n + K) / (2 * K);", "return (2 * h * n + K - 1) / (2 * K);"),
    "presto-odd-harmonics": ("h == 1 || h % 2 == 0;", "h == 1 || h % 2 == 1;"),
    "presto-f32-norm-by-order": ("rs[m - 1], nm[m - 1]", "rs[K - 1], nm[K - 1]"),
    "presto-f64-norm-by-order": ("mu[m - 1]) / sig[m - 1]", "mu[K - 1]) / sig[K - 1]"),
    "presto-stage-one": ("return K >= 2 && (K & (K - 1)) == 0;", "return (K & (K - 1)) == 0;"),
    "presto-first-bin-ignored": ("nearest_bin(1, n, K) < first_bin", "nearest_bin(1, n, K) < 0"),
    "presto-tie-to-larger-stage": ("v > best) { best = v; kb = (int32_t)K; }", "v >= best) { best = v; kb = (int32_t)K; }"),
    "presto-dropped-term": ("S = S + rd32(x, len, nearest_bin(h, n, K));", "S = rd32(x, len, nearest_bin(h, n, K));"),
    "presto-reversed-order": ("rd32(x, len, nearest_bin(h, n, K))", "rd32(x, len, nearest_bin(K + 1 - h, n, K))"),
}

PY_MUTANTS = {
    "sigma-scales-with-k": "import oracle, math\n"
    "_t = oracle.tables\n"
    "def tables(mu1, s1, H):\n"
    "    mu, sig, rs, nm = _t(mu1, s1, H)\n"
    "    import numpy as np\n"
    "    k = np.arange(1, H + 1)\n"
    "    return mu, sig * np.sqrt(k), (1.0 / (sig * np.sqrt(k))).astype(np.float32), (-(mu / (sig * np.sqrt(k)))).astype(np.float32)\n"
    "oracle.tables = tables\n",
    "interbin-amplitude-not-squared": "import oracle, math, numpy as np\n"
    "oracle.INTERBIN_FACTOR = np.float32(math.pi / 4)\n",
    "peak-tie-to-higher-bin": "import oracle, inspect\n"
    "src = inspect.getsource(oracle.cluster_peaks).replace('and j < n', 'and j > n')\n"
    "exec(src, oracle.__dict__)\n",
    "peak-window-one-sided": "import oracle, inspect\n"
    "src = inspect.getsource(oracle.cluster_peaks).replace('min(hi, n + radius + 1)', 'n + 1')\n"
    "exec(src, oracle.__dict__)\n",
    "candidate-at-threshold": "import oracle, inspect\n"
    "src = inspect.getsource(oracle.candidates).replace('snr32 > np.float32(threshold)', 'snr32 >= np.float32(threshold)')\n"
    "exec(src, oracle.__dict__)\n",
    "variance-about-zero": "import oracle\n"
    "_s = oracle.stats\n"
    "def stats(x, first_bin=1):\n"
    "    n, s1, s2 = oracle.exact_sums(x[..., first_bin:])\n"
    "    return float(s1 / n), float(s2 / n)\n"
    "oracle.stats = stats\n",
}


def _run_pins(env, prelude=""):
    code = prelude + "import sys, pytest\nsys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider'] + %r))\n" % PINS
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=600)
    return p.returncode


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_c_mutant_is_caught(name, tmp_path):
    old, new = C_MUTANTS[name]
    src = open(SRC).read()
    assert old in src, "mutation site vanished: " + name
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "mut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-o", str(lib), str(mut), "-lm"],
                   check=True)
    env = dict(os.environ, HS_ORACLE_LIB=str(lib), PYTHONPATH=ROOT + os.pathsep + os.path.join(ROOT, "tests"))
    assert _run_pins(env) != 0, "mutant survived: " + name


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_mutant_is_caught(name):
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.path.join(ROOT, "tests"))
    env.pop("HS_ORACLE_LIB", None)
    assert _run_pins(env, PY_MUTANTS[name]) != 0, "mutant survived: " + name


def test_unmutated_oracle_passes_pins():
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.path.join(ROOT, "tests"))
    env.pop("HS_ORACLE_LIB", None)
    assert _run_pins(env) == 0
