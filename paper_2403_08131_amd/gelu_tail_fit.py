"""Coefficients of the normal tail used by the network kernels (csrc/mlp.hip).

Phi(-a) for a = |u| >= 0 is evaluated as exp2(p(a)) with p a degree-5
polynomial with p(0) = -1 (so Phi(0) = 1/2 exactly), fitted to log2 Phi(-a)
on [0, 6] (beyond, p keeps decreasing from p(6) = -30.25, so the kernels use
it unclamped) so as to minimise the absolute error of Phi(-a): least squares on
Chebyshev points weighted by Phi(-a) (the linearised error), reweighted by
Lawson's iteration towards the minimax fit.  The absolute criterion keeps
the relative error smallest where most activations are, near u = 0, where
a relative error turns directly into bfloat16 rounding flips.  Run this file
to print the coefficients (p_0 .. p_5) and the fit's errors on [0, 6]."""
import numpy as np
from scipy.special import log_ndtr

A = 6.0
DEG = 5


def fit(iterations=80):
    a = 0.5 * A * (1.0 - np.cos(np.linspace(0.0, np.pi, 6000)))
    f = log_ndtr(-a) / np.log(2.0)
    phi = np.exp2(f)
    V = np.vander(a, DEG + 1, increasing=True)[:, 1:]  # p(a) = -1 + a q(a)
    w = np.ones_like(a)
    for _ in range(iterations):
        s = np.sqrt(w) * phi
        q, *_ = np.linalg.lstsq(V * s[:, None], (f + 1.0) * s, rcond=None)
        c = np.concatenate([[-1.0], q])
        e = np.abs(np.exp2(np.polynomial.polynomial.polyval(a, c)) - phi)
        w = w * e
        w /= w.sum()
    return c


def errors(c):
    aa = np.linspace(0.0, A, 400001)
    exact = np.exp(log_ndtr(-aa))
    approx = np.exp2(np.polynomial.polynomial.polyval(aa, c))
    rel_small = np.max(np.abs(approx / exact - 1.0)[aa <= 1.0])
    return np.max(np.abs(approx - exact)), rel_small, np.max(np.abs(aa * (approx - exact)))


if __name__ == "__main__":
    c = fit()
    for i, v in enumerate(c):
        print(f"p{i} = {float(np.float32(v))!r}f")
    print("max absolute error of Phi(-a): %.3g, relative on [0, 1]: %.3g, "
          "absolute of a Phi(-a): %.3g" % errors(c))
