"""The normal tail of the network kernels: the coefficients written in
csrc/mlp.hip, evaluated in float32 in the kernel's order (Horner, then
exp2), reproduce Phi(-a) on [0, 6] within the stated bounds against scipy's
log_ndtr (absolute error <= 5e-7, relative error <= 5e-6 for a <= 1,
Phi(0) = 1/2 exactly); beyond 6, where the kernel takes the polynomial
unclamped, its float32 value keeps decreasing (tail below its value at 6,
within 5e-7 of Phi(-a), 0 for huge or infinite a, never NaN); they are the
ones gelu_tail_fit.py computes; and the prescreen's doubled GELU uses the
same polynomial with its constant raised by 1 (2 Phi(-a) = exp2(p(a) + 1))."""
import os
import re

import numpy as np
from scipy.special import log_ndtr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _coefficients():
    src = open(os.path.join(ROOT, "paper_2403_08131_amd", "csrc", "mlp.hip")).read()
    body = src[src.index("float normal_tail(float u)"):]
    body = body[:body.index("return __builtin_amdgcn_exp2f(p);")]
    lits = [float(v) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    # |u| unclamped, then the two highest coefficients in the first fma, then
    # the rest down to the constant
    assert "fminf" not in body and len(lits) == 6
    return [np.float32(v) for v in lits]  # highest degree first


def _poly32(a):
    c = _coefficients()
    m = np.abs(np.asarray(a, dtype=np.float32))
    with np.errstate(over="ignore", invalid="ignore"):
        p = (np.float32(c[0]) * m + np.float32(c[1])).astype(np.float32)
        for v in c[2:]:
            p = (p * m + v).astype(np.float32)
    return p


def _tail32(a):
    return np.exp2(_poly32(a).astype(np.float64))


def test_tail_within_bound():
    a = np.linspace(0.0, 6.0, 200001).astype(np.float32)
    exact = np.exp(log_ndtr(-a.astype(np.float64)))
    t = _tail32(a)
    assert np.max(np.abs(t - exact)) <= 5e-7
    assert np.max(np.abs(t / exact - 1.0)[a <= 1.0]) <= 5e-6
    assert _tail32(np.float32(0.0)) == 0.5
    assert _tail32(np.float32(6.0)) < 1e-8


def test_tail_beyond_the_fit_interval():
    a = np.linspace(6.0, 1e4, 2000001).astype(np.float32)
    p = _poly32(a)
    assert np.all(np.diff(p) <= 0)
    t = _tail32(a)
    assert np.all(t <= _tail32(np.float32(6.0)))
    exact = np.exp(log_ndtr(-a.astype(np.float64)))
    assert np.max(np.abs(t - exact)) <= 5e-7
    huge = np.array([1e7, 1e20, 3.4e38, np.inf], dtype=np.float32)
    p = _poly32(huge)
    assert not np.any(np.isnan(p)) and np.all(_tail32(huge) == 0.0)


def test_coefficients_match_the_fit():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "gelu_tail_fit", os.path.join(ROOT, "paper_2403_08131_amd", "gelu_tail_fit.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    c = mod.fit()
    np.testing.assert_array_equal(np.float32(c[::-1]), np.array(_coefficients(), dtype=np.float32))


def test_doubled_gelu_uses_the_same_polynomial():
    src = open(os.path.join(ROOT, "paper_2403_08131_amd", "csrc", "mlp.hip")).read()
    body = src[src.index("float gelu2(float u)"):]
    body = body[:body.index("return fmaf(")]
    lits = [np.float32(float(v)) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    c = _coefficients()
    assert lits == c[:-1] and c[-1] == np.float32(-1.0)
    assert "p = m * p;" in body  # the constant term p(0) + 1 = 0
