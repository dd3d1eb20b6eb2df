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
    "append_back_sub": ("oracle_forward_sub(n, L, k, l);", "oracle_back_sub(n, L, k, l);"),
    "append_no_sqrt": ("Lout[(size_t)n * n1 + n] = sqrt(d2);", "Lout[(size_t)n * n1 + n] = d2;"),
    "grad_double": ("grad[k] += 0.5 * w * dr * t * t;", "grad[k] += w * dr * t * t;"),
    "grad_kinv_sign": ("const double w = alpha[i] * alpha[l] - Kinv[(size_t)i * n + l];",
                       "const double w = alpha[i] * alpha[l] + Kinv[(size_t)i * n + l];"),
    "grad_matern_drop": ("dr = sf2 * (5.0 / 3.0) * (1.0 + sqrt(5.0) * r) * exp(-sqrt(5.0) * r);",
                         "dr = sf2 * (5.0 / 3.0) * exp(-sqrt(5.0) * r);"),
    "grad_noise_sf2": ("if (i == l) grad[d + 1] += 0.5 * w * sn2;",
                       "if (i == l) grad[d + 1] += 0.5 * w * sf2;"),
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


PLAN_MUTATIONS = {
    "sens_no_abs": ("acc += abs((base[r] - out[j, i, r]) / base[r])",
                    "acc += (base[r] - out[j, i, r]) / base[r]"),
    "sens_no_mean": ("S[r, j] = acc / V", "S[r, j] = acc"),
    "influence_min": ("top = max(own) if own else 0.0", "top = min(own) if own else 0.0"),
    "cut_below": ("if r != o and I[r, j] >= cutoff:", "if r != o and I[r, j] <= cutoff:"),
    "cap_smallest": ("key=lambda j: (-score[j], j)", "key=lambda j: (score[j], j)"),
    "merge_one_way": ("                adj[r].add(o)\n", ""),
}


@pytest.mark.slow
def test_plan_pins_catch_planted_mistakes():
    """The same check for the planning oracle (oracle/plan.py): each planted
    mistake must fail a pin of tests/test_oracle_plan.py."""
    src = os.path.join(ROOT, "oracle", "plan.py")
    with open(src) as f:
        text = f.read()
    pins = os.path.join(ROOT, "tests", "test_oracle_plan.py")
    survivors = []
    with tempfile.TemporaryDirectory() as tmp:
        for name, (old, new) in list(PLAN_MUTATIONS.items()) + [("clean", ("", ""))]:
            pkg = os.path.join(tmp, name, "oracle")
            os.makedirs(pkg)
            open(os.path.join(pkg, "__init__.py"), "w").close()
            if name != "clean":
                assert text.count(old) >= 1, name
            with open(os.path.join(pkg, "plan.py"), "w") as f:
                f.write(text.replace(old, new, 1) if name != "clean" else text)
            env = dict(os.environ, PYTHONPATH=os.path.join(tmp, name) + os.pathsep + ROOT)
            r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                                "--rootdir", os.path.join(tmp, name), pins],
                               cwd=os.path.join(tmp, name), env=env, capture_output=True, text=True,
                               timeout=600)
            if name == "clean":
                assert r.returncode == 0, r.stdout[-2000:]
            elif r.returncode == 0:
                survivors.append(name)
    assert not survivors, f"plan pins did not catch: {survivors}"


BO_MUTATIONS = {
    "pick_argmin": ("j = O.argmax(ei)", "j = int(np.argmin(ei))"),
    "pick_first_row": ("x = P[j].copy()", "x = P[0].copy()"),
    "no_normalize": ("f = O.fit(X, y, ls, kind, sf2, sn2, normalize_y)",
                     "f = O.fit(X, y, ls, kind, sf2, sn2, False)"),
    "stale_objective": ("y = np.append(y, float(objective(x)))",
                        "y = np.append(y, float(objective(P[0])))"),
    "fit_initial_only": ("f = O.fit(X, y, ls, kind, sf2, sn2, normalize_y)",
                         "f = O.fit(X[:len(X0)], y[:len(X0)], ls, kind, sf2, sn2, normalize_y)"),
}


def _python_survivors(module, pins_file, mutations):
    """Plant each mutation in a copy of oracle/<module> (the rest of the
    oracle package linked in) and run the pins; returns the mutations no pin
    caught (the unaltered copy must pass)."""
    src = os.path.join(ROOT, "oracle", module)
    with open(src) as f:
        text = f.read()
    pins = os.path.join(ROOT, "tests", pins_file)
    survivors = []
    with tempfile.TemporaryDirectory() as tmp:
        for name, (old, new) in list(mutations.items()) + [("clean", ("", ""))]:
            pkg = os.path.join(tmp, name, "oracle")
            os.makedirs(pkg)
            open(os.path.join(pkg, "__init__.py"), "w").close()
            for aux in ("oracle.py", "gp_oracle.c", "liboracle.so"):
                os.symlink(os.path.join(ROOT, "oracle", aux), os.path.join(pkg, aux))
            if name != "clean":
                assert text.count(old) >= 1, name
            with open(os.path.join(pkg, module), "w") as f:
                f.write(text.replace(old, new, 1) if name != "clean" else text)
            env = dict(os.environ, PYTHONPATH=os.path.join(tmp, name) + os.pathsep + ROOT)
            r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                                "--rootdir", os.path.join(tmp, name), pins],
                               cwd=os.path.join(tmp, name), env=env, capture_output=True, text=True,
                               timeout=600)
            if name == "clean":
                assert r.returncode == 0, r.stdout[-2000:]
            elif r.returncode == 0:
                survivors.append(name)
    return survivors


@pytest.mark.slow
def test_bo_pins_catch_planted_mistakes():
    """The same check for the loop oracle (oracle/bo.py) and its pins in
    tests/test_oracle_bo.py."""
    survivors = _python_survivors("bo.py", "test_oracle_bo.py", BO_MUTATIONS)
    assert not survivors, f"bo pins did not catch: {survivors}"


HYPER_MUTATIONS = {
    "adam_descent": ("th = np.clip(th + lr * mh", "th = np.clip(th - lr * mh"),
    "no_bias_correction": ("mh = m / (1.0 - beta1 ** t)", "mh = m"),
    "jitter_starts_high": ("sf2 * jitter0 * 10.0 ** (k - 1)", "sf2 * jitter0 * 10.0 ** k"),
    "noise_grad_unscaled": ("g[d + 1] *= sn2 / (sn2 + jit)", "g[d + 1] *= 1.0"),
    "best_is_min": ('if r["lml"] > res[best]["lml"]:', 'if r["lml"] < res[best]["lml"]:'),
}


@pytest.mark.slow
def test_hyper_pins_catch_planted_mistakes():
    """The same check for the hyperparameter-fitting oracle (oracle/hyper.py)
    and its pins in tests/test_oracle_hyper.py."""
    survivors = _python_survivors("hyper.py", "test_oracle_hyper.py", HYPER_MUTATIONS)
    assert not survivors, f"hyper pins did not catch: {survivors}"
