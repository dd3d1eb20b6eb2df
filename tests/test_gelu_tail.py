"""The normal tail of the network kernels: the coefficients written in
csrc/mlp.hip, evaluated in float32 in the kernel's order (Horner, then
exp2), reproduce Phi(-a) on [0, 6] within the stated bounds against scipy's
log_ndtr (absolute error <= 5e-7, relative error <= 5e-6 for a <= 1,
Phi(0) = 1/2 exactly) and stay at their value at 6 beyond; and they are the
ones gelu_tail_fit.py computes."""
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
    # min(|u|, 6.0f), then the two highest coefficients in the first fma,
    # then the rest down to the constant
    assert lits[0] == 6.0
    return [np.float32(v) for v in lits[1:]]  # highest degree first


def _tail32(a):
    c = _coefficients()
    m = np.minimum(np.abs(a), np.float32(6.0)).astype(np.float32)
    p = np.float32(c[0]) * m + np.float32(c[1])
    for v in c[2:]:
        p = (p * m + v).astype(np.float32)
    return np.exp2(p.astype(np.float64))


def test_tail_within_bound():
    a = np.linspace(0.0, 6.0, 200001).astype(np.float32)
    exact = np.exp(log_ndtr(-a.astype(np.float64)))
    t = _tail32(a)
    assert np.max(np.abs(t - exact)) <= 5e-7
    assert np.max(np.abs(t / exact - 1.0)[a <= 1.0]) <= 5e-6
    assert _tail32(np.float32(0.0)) == 0.5
    big = np.array([6.0, 7.5, 40.0], dtype=np.float32)
    assert np.allclose(_tail32(big), _tail32(np.float32(6.0)), rtol=0, atol=0)
    assert _tail32(np.float32(6.0)) < 1e-8


def test_coefficients_match_the_fit():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "gelu_tail_fit", os.path.join(ROOT, "paper_2403_08131_amd", "gelu_tail_fit.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    c = mod.fit()
    np.testing.assert_array_equal(np.float32(c[::-1]), np.array(_coefficients(), dtype=np.float32))
