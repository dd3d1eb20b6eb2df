"""The oracle's pins catch plausible slips.

Each case copies ``oracle/gp_oracle.c``, plants one mistake in the copy (a
dropped term, a wrong sign, a transposed index, ...), builds it on the CPU
and runs the pin suite against that build in a subprocess.  The pins must
fail for every planted mistake, and pass for the unaltered source.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gp_oracle.c")

MUTATIONS = {
    "se_drop_half": ("exp(-0.5 * r2)", "exp(-r2)"),
    "matern_coef": ("5.0 * r2 / 3.0", "5.0 * r2 / 2.0"),
    "chol_sign": ("s -= L[(size_t)i * n + k] * L[(size_t)j * n + k]",
                  "s += L[(size_t)i * n + k] * L[(size_t)j * n + k]"),
    "chol_index": ("s -= L[(size_t)i * n + k] * L[(size_t)j * n + k]",
                   "s -= L[(size_t)i * n + k] * L[(size_t)k * n + j]"),
    "backsub_transposed": ("s -= L[(size_t)k * n + i] * x[k]", "s -= L[(size_t)i * n + k] * x[k]"),
    "lml_drop_logdet": ("-0.5 * quad - 0.5 * logdet", "-0.5 * quad"),
    "var_drop_sf2": ("double varz = sf2 - vv;", "double varz = 1.0 - vv;"),
    "mean_drop_scale": ("double mj = ymean + sy * muz;", "double mj = ymean + muz;"),
    "sample_std": ("var /= n;", "var /= (n - 1);"),
    "ei_sign": ("double imp = fbest - mu;", "double imp = mu - fbest;"),
    "ei_cdf_sign": ("0.5 * erfc(-z / sqrt(2.0))", "0.5 * erfc(z / sqrt(2.0))"),
    "gelu_grad_drop": ("+ u * exp(-0.5 * u * u) / sqrt(2.0 * OR_PI)", ""),
    "adam_no_bias_corr": ("double mh = m[i] / c1;", "double mh = m[i];"),
    "bf16_round_half_up": ("u = (u + 0x7fffu + lsb) & 0xffff0000u;", "u = (u + 0x8000u) & 0xffff0000u;"),
    "argmax_last_tie": ("if (best < 0 || v[j] > v[best]) best = j;\n  }\n  return best;",
                        "if (best < 0 || v[j] >= v[best]) best = j;\n  }\n  return best;"),
    "ens_sample_std": ("sqrt(q / E)", "sqrt(q / (E - 1))"),
    "bound_drop_noise": ("kmax * kmax / (sf2 + sn2)", "kmax * kmax / sf2"),
    "bound_min_k": ("if (k > kmax) kmax = k;", "if (kmax == 0.0 || k < kmax) kmax = k;"),
    "w2_transposed": ("s += rnd(W2[(size_t)h * H + k], bf16) * h1[k];",
                      "s += rnd(W2[(size_t)k * H + h], bf16) * h1[k];"),
}


def _build(src_text, out):
    cpath = out + ".c"
    with open(cpath, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                           "-fno-fast-math", "-ffp-contract=off", cpath, "-o", out, "-lm"])


def _run_pins(lib_path):
    env = dict(os.environ, GPBO_ORACLE_LIB=lib_path, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not slow",
                        "-p", "no:cacheprovider", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode


@pytest.mark.slow
def test_pins_catch_planted_mistakes():
    with open(SRC) as f:
        text = f.read()
    with tempfile.TemporaryDirectory() as tmp:
        jobs = {}
        for name, (old, new) in MUTATIONS.items():
            assert text.count(old) >= 1, name
            mutated = text.replace(old, new, 1)
            out = os.path.join(tmp, f"lib_{name}.so")
            _build(mutated, out)
            jobs[name] = out
        clean = os.path.join(tmp, "lib_clean.so")
        _build(text, clean)
        with ThreadPoolExecutor(max_workers=4) as ex:
            codes = dict(zip(list(jobs) + ["clean"],
                             ex.map(_run_pins, list(jobs.values()) + [clean])))
    assert codes.pop("clean") == 0
    survivors = [k for k, c in codes.items() if c == 0]
    assert not survivors, f"pins did not catch: {survivors}"
