"""Pins of the hyperparameter-fitting oracle (oracle/hyper.py): each step is
the Adam update of the separately pinned LML gradient, the LML rises from
the start on well-posed data, the returned optimum is stationary by central
differences of the LML, data drawn from a Gaussian process with known
hyperparameters give them back within their sampling spread, the best start
is the one with the largest final LML, and a singular K takes the jitter
path."""
import math

import numpy as np

from oracle import hyper as H
from oracle import oracle as O

LO = np.log([1e-2, 1e-2, 1e-3, 1e-6])
HI = np.log([1e2, 1e2, 1e2, 1.0])


def _data(seed, n=40):
    rng = np.random.default_rng(seed)
    X = rng.uniform(size=(n, 2))
    y = np.sin(6.0 * X[:, 0]) + 0.5 * X[:, 1] + 0.05 * rng.standard_normal(n)
    return X, y


def test_first_steps_are_adam_updates_of_the_gradient():
    X, y = _data(1)
    th0 = np.log([0.5, 0.5, 1.0, 1e-2])
    r = H.fit_start(X, y, th0, LO, HI, O.SE, steps=3, lr=0.05)
    th, m, v = th0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 4):
        st, g, _ = O.lml_grad(X, y, np.exp(th[:2]), O.SE, math.exp(th[2]), math.exp(th[3]))
        assert st == O.OK
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        th = np.clip(th + 0.05 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8), LO, HI)
        np.testing.assert_allclose(r["path"][t - 1], th, rtol=0, atol=1e-14)


def test_lml_rises_and_optimum_is_stationary():
    X, y = _data(2)
    r = H.fit_start(X, y, np.log([0.3, 2.0, 0.5, 1e-1]), LO, HI, O.SE, steps=400, lr=0.05)
    assert r["alive"] and r["jitter"] == 0.0
    assert r["lml"] > r["lml0"] + 1.0
    th = r["theta"]
    interior = (th > LO + 0.1) & (th < HI - 0.1)

    def lml(t):
        return O.fit(X, y, np.exp(t[:2]), O.SE, math.exp(t[2]), math.exp(t[3])).lml

    h = 1e-5
    fd = np.array([(lml(th + h * e) - lml(th - h * e)) / (2 * h) for e in np.eye(4)])
    assert np.all(np.abs(fd[interior]) < 0.05 * max(1.0, abs(r["lml"]) / len(y))), fd


def test_recovers_hyperparameters_of_gp_draws():
    """200 points of a 1-d GP draw (SE, l = 0.2, sf2 = 1, sn2 = 0.01) give
    the lengthscale within 25 % and the noise variance within a factor 2."""
    rng = np.random.default_rng(9)
    X = rng.uniform(size=(200, 1))
    K = O.gram(O.SE, X, [0.2], 1.0, 0.01)
    y = np.linalg.cholesky(K) @ rng.standard_normal(200)
    lo, hi = np.log([1e-2, 1e-3, 1e-6]), np.log([1e2, 1e2, 1.0])
    best, res = H.fit(X, y, [np.log([0.5, 0.5, 0.1]), np.log([0.05, 2.0, 1e-3])], lo, hi, O.SE,
                      steps=300, lr=0.05, normalize_y=False)
    th = res[best]["theta"]
    assert abs(math.exp(th[0]) / 0.2 - 1.0) < 0.25, np.exp(th)
    assert 0.5 < math.exp(th[2]) / 0.01 < 2.0, np.exp(th)
    assert res[best]["lml"] == max(r["lml"] for r in res)


def test_singular_kernel_matrix_takes_the_jitter_path():
    """Two identical points, SE, sf2 = 1, sn2 = 1e-30: K = [[1, 1], [1, 1]]
    in float64, the second pivot is exactly 0; the first jitter (1e-8)
    makes it positive."""
    X = np.array([[0.2, 0.4], [0.2, 0.4], [0.9, 0.1]])
    y = np.array([0.0, 0.1, 1.0])
    th = np.log([0.3, 0.3, 1.0, 1e-30])
    st, g, lml, jit = H.lml_grad_jitter(X, y, th, O.SE)
    assert st == O.OK and jit == 1e-8 and np.isfinite(lml)
    st0, _, _ = O.lml_grad(X, y, [0.3, 0.3], O.SE, 1.0, 1e-30)
    assert st0 == O.NOT_PD
    # the log-noise derivative is that of sn2 itself: scaled by sn2 / (sn2 + jitter)
    sn2 = math.exp(th[3])
    _, g_j, _ = O.lml_grad(X, y, np.exp(th[:2]), O.SE, 1.0, sn2 + 1e-8)
    assert g[3] == g_j[3] * (sn2 / (sn2 + 1e-8))
