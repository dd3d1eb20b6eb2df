"""Pins of the Bayesian-optimisation loop oracle (oracle/bo.py) against what
the loop's definition fixes: every pick is the argmax of an expected
improvement computed by an independent route (dense LU solves of K, the
normal distribution from scipy), the evaluated set grows by exactly the
picked rows with their objective values, the best value never rises, and a
one-dimensional search whose pool holds the objective's minimiser finds it."""
import numpy as np
import pytest
import scipy.stats

from oracle import bo as BO
from oracle import oracle as O

SF2, SN2 = 1.0, 1e-4


def _objective(x):
    x = np.asarray(x, dtype=np.float64)
    return float(np.sum((x - 0.3) ** 2) + 0.5 * np.sin(7.0 * x[0]))


def _case(d, n_init, iters, m, seed, kind=O.SE):
    rng = np.random.default_rng(seed)
    X0 = rng.uniform(size=(n_init, d))
    y0 = np.array([_objective(x) for x in X0])
    pools = [rng.uniform(size=(m, d)) for _ in range(iters)]
    ls = np.full(d, 0.35)
    return X0, y0, pools, ls, kind


def _dense_ei(X, y, P, ls, kind):
    """EI of the pool by LU solves of K (no Cholesky) and scipy's normal."""
    n = X.shape[0]
    mean, sy = y.mean(), y.std()
    sy = sy if sy > 0 else 1.0
    yt = (y - mean) / sy
    K = O.gram(kind, X, ls, SF2, SN2)
    Kall = O.gram(kind, np.vstack([X, P]), ls, SF2, 0.0)
    Ks = Kall[n:, :n]
    mu = mean + sy * Ks @ np.linalg.solve(K, yt)
    var = SF2 - np.einsum("ij,ji->i", Ks, np.linalg.solve(K, Ks.T))
    sd = sy * np.sqrt(np.maximum(var, 0.0))
    imp = y.min() - mu
    z = imp / sd
    return imp * scipy.stats.norm.cdf(z) + sd * scipy.stats.norm.pdf(z)


@pytest.mark.parametrize("d,kind,seed", [(2, O.SE, 1), (3, O.MATERN52, 2)])
def test_picks_are_argmax_of_independent_ei(d, kind, seed):
    X0, y0, pools, ls, kind = _case(d, 5, 8, 96, seed, kind)
    r = BO.search(_objective, X0, y0, pools, ls, kind, SF2, SN2)
    for t, P in enumerate(pools):
        n = X0.shape[0] + t
        ei = _dense_ei(r["X"][:n], r["y"][:n], P, ls, kind)
        assert r["picks"][t] == int(np.argmax(ei)), t
        np.testing.assert_allclose(r["ei_max"][t], ei.max(), rtol=1e-8, atol=1e-14)


def test_evaluated_set_grows_by_the_picks():
    X0, y0, pools, ls, kind = _case(2, 5, 6, 50, 7)
    r = BO.search(_objective, X0, y0, pools, ls, kind, SF2, SN2)
    assert r["X"].shape == (5 + 6, 2) and r["y"].shape == (11,)
    np.testing.assert_array_equal(r["X"][:5], X0)
    for t, P in enumerate(pools):
        np.testing.assert_array_equal(r["X"][5 + t], P[r["picks"][t]])
    np.testing.assert_array_equal(r["y"], [_objective(x) for x in r["X"]])


def test_best_value_never_rises():
    X0, y0, pools, ls, kind = _case(3, 5, 10, 64, 11)
    r = BO.search(_objective, X0, y0, pools, ls, kind, SF2, SN2)
    fb = np.array(r["fbest"])
    assert np.all(np.diff(fb) <= 0.0)
    for t in range(len(pools)):
        assert fb[t] == r["y"][: 5 + t + 1].min()


def test_one_dimensional_search_finds_pool_minimiser():
    grid = np.linspace(0.0, 1.0, 101)[:, None]
    f = lambda x: float((x[0] - 0.3) ** 2)
    rng = np.random.default_rng(5)
    X0 = rng.uniform(size=(5, 1))
    y0 = np.array([f(x) for x in X0])
    r = BO.search(f, X0, y0, [grid] * 15, [0.2], O.SE, SF2, SN2)
    assert min(r["y"]) == 0.0 or abs(r["X"][int(np.argmin(r["y"]))][0] - 0.3) < 1e-12
