"""Pins of the float64 oracle against what mathematics and the paper fix.

Each test checks the oracle against something other than itself: closed
forms, brute force at tiny sizes, library special cases (numpy / scipy /
torch, used here only), Monte Carlo, finite differences and hand values under
``tests/golden/``.  A plausible slip anywhere in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.special
import scipy.stats

from oracle import oracle as O
from paper_2403_08131_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# Covariance functions
# ---------------------------------------------------------------------------

def test_kernel_golden_values():
    g = _golden("kernel_values.json")
    a = np.zeros(1)
    b = np.ones(1)
    assert O.kernel(O.SE, a, b, [1.0]) == pytest.approx(g["se_r1"], abs=1e-15)
    assert O.kernel(O.MATERN52, a, b, [1.0]) == pytest.approx(g["matern52_r1"], abs=1e-6)
    # SE at distance equal to the lengthscale, one dimension, with a signal variance
    assert O.kernel(O.SE, [0.3], [0.3 + 0.7], [0.7], 2.5) == pytest.approx(2.5 * math.exp(-0.5), rel=1e-15)


@pytest.mark.parametrize("kind", [O.SE, O.MATERN52])
def test_kernel_diagonal_and_symmetry(kind):
    r = _rng(1)
    ls = r.uniform(0.1, 2.0, 5)
    a, b = r.uniform(0, 1, 5), r.uniform(0, 1, 5)
    assert O.kernel(kind, a, a, ls, 1.7) == 1.7
    assert O.kernel(kind, a, b, ls, 1.7) == O.kernel(kind, b, a, ls, 1.7)


def test_matern52_matches_general_matern_bessel():
    """Matern-5/2 closed form vs the general Matern with a modified Bessel
    function (R&W eq. 4.14), nu = 5/2, through scipy.special.kv."""
    nu = 2.5
    for r in [0.05, 0.3, 1.0, 2.2, 4.0]:
        t = math.sqrt(2 * nu) * r
        general = 2 ** (1 - nu) / scipy.special.gamma(nu) * t ** nu * scipy.special.kv(nu, t)
        assert O.kernel(O.MATERN52, [0.0], [r], [1.0]) == pytest.approx(general, rel=1e-12)


@pytest.mark.parametrize("kind", [O.SE, O.MATERN52])
def test_kernel_ard_lengthscale_per_dimension(kind):
    """Per-dimension lengthscales: doubling l_k is the same as halving the k-th
    coordinate difference, and each dimension enters separately."""
    r = _rng(2)
    a, b = r.uniform(0, 1, 4), r.uniform(0, 1, 4)
    ls = np.array([0.3, 0.5, 0.7, 1.1])
    ls2 = ls.copy()
    ls2[2] *= 2
    b2 = b.copy()
    b2[2] = a[2] + (b[2] - a[2]) / 2
    assert O.kernel(kind, a, b, ls2) == pytest.approx(O.kernel(kind, a, b2, ls), rel=1e-14)
    # SE factorises over dimensions
    if kind == O.SE:
        prod = 1.0
        for k in range(4):
            prod *= math.exp(-0.5 * ((a[k] - b[k]) / ls[k]) ** 2)
        assert O.kernel(kind, a, b, ls) == pytest.approx(prod, rel=1e-14)


@pytest.mark.parametrize("kind", [O.SE, O.MATERN52])
def test_gram_symmetric_pd_with_noise_on_diagonal(kind):
    r = _rng(3)
    X = r.uniform(0, 1, (12, 3))
    ls = [0.4, 0.6, 0.9]
    K = O.gram(kind, X, ls, 1.3, 0.05)
    assert np.array_equal(K, K.T)
    assert np.allclose(np.diag(K), 1.3 + 0.05, rtol=0, atol=1e-15)
    assert K[3, 7] == O.kernel(kind, X[3], X[7], ls, 1.3)
    assert np.linalg.eigvalsh(K).min() > 0


# ---------------------------------------------------------------------------
# Cholesky, solves, log determinant, log marginal likelihood
# ---------------------------------------------------------------------------

def _spd(n, seed):
    r = _rng(seed)
    A = r.normal(size=(n, n))
    return A @ A.T + n * np.eye(n)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_cholesky_brute_force_product(n):
    K = _spd(n, n)
    st, L, bad = O.cholesky(K)
    assert st == O.OK and bad == -1
    assert np.all(np.triu(L, 1) == 0)
    assert np.all(np.diag(L) > 0)
    P = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            P[i, j] = sum(L[i, k] * L[j, k] for k in range(n))
    assert np.abs(P - K).max() <= 1e-14 * np.abs(K).max() * n


def test_cholesky_library_special_case():
    K = _spd(40, 7)
    st, L, _ = O.cholesky(K)
    assert st == O.OK
    assert np.allclose(L, np.linalg.cholesky(K), rtol=1e-13, atol=1e-13)


def test_cholesky_not_pd_reports_pivot():
    # duplicate rows with no noise: the second copy's pivot is exactly zero
    X = np.array([[0.1, 0.2], [0.5, 0.9], [0.1, 0.2], [0.7, 0.3]])
    K = O.gram(O.SE, X, [0.5, 0.5], 1.0, 0.0)
    st, _, bad = O.cholesky(K)
    assert st == O.NOT_PD and bad == 2
    K2 = np.eye(3)
    K2[0, 0] = -1.0
    st, _, bad = O.cholesky(K2)
    assert st == O.NOT_PD and bad == 0
    K3 = np.eye(3)
    K3[1, 1] = np.nan
    st, _, bad = O.cholesky(K3)
    assert st == O.NOT_PD and bad == 1


@pytest.mark.parametrize("n", [0, 1, 7, 33])
@pytest.mark.parametrize("kind", [O.SE, O.MATERN52])
def test_chol_append_equals_factor_of_bordered_matrix(n, kind):
    """The Cholesky factor with positive diagonal is unique, so extending the
    factor of K by one row must give the factor of the bordered matrix."""
    rng = np.random.default_rng(300 + n + 10 * kind)
    X = rng.uniform(size=(n + 1, 3))
    K = O.gram(kind, X, [0.4, 0.7, 1.1], 1.3, 1e-3)
    st, Lf, _ = O.cholesky(K)
    assert st == O.OK
    L = Lf[:n, :n] if n else np.zeros((0, 0))
    st, La, bad = O.chol_append(L, K[n, :n], K[n, n])
    assert st == O.OK and bad == -1
    np.testing.assert_allclose(La, Lf, rtol=0, atol=1e-13)
    np.testing.assert_allclose(La @ La.T, K, rtol=0, atol=1e-13)
    assert np.all(np.triu(La, 1) == 0.0)


def test_chol_append_n0_is_sqrt_and_not_pd_reports_new_index():
    st, La, _ = O.chol_append(np.zeros((0, 0)), np.zeros(0), 6.25)
    assert st == O.OK and La.shape == (1, 1) and La[0, 0] == 2.5
    # bordered matrix [[4, 2], [2, 0.5]] has determinant -2: not positive definite
    st, _, bad = O.chol_append(np.array([[2.0]]), np.array([2.0]), 0.5)
    assert st == O.NOT_PD and bad == 1
    # [[4, 2], [2, 1]] is singular: the new pivot is exactly zero
    st, _, bad = O.chol_append(np.array([[2.0]]), np.array([2.0]), 1.0)
    assert st == O.NOT_PD and bad == 1
    # [[4, 2], [2, 2]]: l = 1, delta = 1
    st, La, _ = O.chol_append(np.array([[2.0]]), np.array([2.0]), 2.0)
    assert st == O.OK and np.array_equal(La, np.array([[2.0, 0.0], [1.0, 1.0]]))


@pytest.mark.parametrize("kind", [O.SE, O.MATERN52])
@pytest.mark.parametrize("normalize", [True, False])
def test_lml_gradient_central_differences(kind, normalize):
    """dLML/dlog(theta) against central differences of the (separately pinned)
    log marginal likelihood, including the noise and signal terms."""
    rng = np.random.default_rng(71 + kind)
    X = rng.uniform(size=(14, 3))
    y = np.sin(4.0 * X[:, 0]) + X[:, 1] ** 2 + 0.1 * rng.standard_normal(14)
    th = np.log([0.4, 0.7, 1.1, 1.3, 2e-2])

    def lml(t):
        return O.fit(X, y, np.exp(t[:3]), kind, np.exp(t[3]), np.exp(t[4]), normalize).lml

    st, g, l0 = O.lml_grad(X, y, np.exp(th[:3]), kind, np.exp(th[3]), np.exp(th[4]), normalize)
    assert st == O.OK and l0 == lml(th)
    h = 1e-5
    fd = np.array([(lml(th + h * e) - lml(th - h * e)) / (2 * h) for e in np.eye(5)])
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_lml_gradient_n1_closed_form():
    """n = 1, centred only: LML = -y~^2 / (2 s) - log(s) / 2 - log(2 pi) / 2 with
    s = sf2 + sn2 and y~ = 0, so dLML/dlog sf2 = -sf2 / (2 s), dLML/dlog sn2 =
    -sn2 / (2 s), and the lengthscales do not enter."""
    st, g, l0 = O.lml_grad(np.array([[0.3, 0.9]]), np.array([2.0]), [0.5, 0.5], O.SE, 1.5, 0.5,
                           False)
    assert st == O.OK
    np.testing.assert_allclose(g, [0.0, 0.0, -1.5 / 4.0, -0.5 / 4.0], rtol=1e-15, atol=0)
    assert l0 == pytest.approx(-0.5 * np.log(2.0) - 0.5 * np.log(2 * np.pi), rel=1e-15)


def test_triangular_solves_residual():
    K = _spd(9, 11)
    _, L, _ = O.cholesky(K)
    b = _rng(5).normal(size=9)
    z = O.forward_sub(L, b)
    assert np.abs(L @ z - b).max() < 1e-13
    x = O.back_sub(L, z)
    assert np.abs(L.T @ x - z).max() < 1e-13
    assert np.abs(K @ x - b).max() < 1e-12 * np.abs(b).max() * np.linalg.cond(K)


def _leibniz_det(A):
    n = A.shape[0]
    total = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        p = 1.0
        for i in range(n):
            p *= A[i, perm[i]]
        total += (-1) ** inv * p
    return total


@pytest.mark.parametrize("n", [1, 3, 6, 8])
def test_logdet_brute_force_determinant(n):
    r = _rng(20 + n)
    X = r.uniform(0, 1, (n, 2))
    y = r.normal(size=n)
    f = O.fit(X, y, [0.3, 0.6], O.SE, 1.0, 0.1)
    assert f.status == O.OK
    K = O.gram(O.SE, X, [0.3, 0.6], 1.0, 0.1)
    assert f.logdet == pytest.approx(math.log(_leibniz_det(K)), rel=1e-12, abs=1e-12)


def test_lml_n1_closed_form():
    # n = 1: ytilde = 0 after centring, so test with normalisation off
    sf2, sn2 = 1.4, 0.3
    y = np.array([0.8])
    f = O.fit(np.array([[0.2, 0.4]]), y, [0.5, 0.5], O.SE, sf2, sn2, normalize_y=False)
    # centre only: ytilde = y - mean(y) = 0
    s = sf2 + sn2
    assert f.lml == pytest.approx(-0.5 * math.log(2 * math.pi * s), rel=1e-14)


def test_lml_against_multivariate_normal():
    r = _rng(4)
    n = 25
    X = r.uniform(0, 1, (n, 3))
    y = r.normal(size=n) * 3 + 1
    for kind in (O.SE, O.MATERN52):
        f = O.fit(X, y, [0.4, 0.5, 0.6], kind, 1.2, 0.02)
        K = O.gram(kind, X, [0.4, 0.5, 0.6], 1.2, 0.02)
        yt = (y - y.mean()) / y.std()
        ref = scipy.stats.multivariate_normal(mean=np.zeros(n), cov=K).logpdf(yt)
        assert f.lml == pytest.approx(ref, rel=1e-11)
        assert f.ymean == pytest.approx(y.mean(), rel=1e-15)
        assert f.ystd == pytest.approx(y.std(), rel=1e-14)
        assert f.fbest == y.min()


def test_alpha_n2_explicit_inverse_and_residual():
    X = np.array([[0.1, 0.3], [0.6, 0.2]])
    y = np.array([1.0, -2.0])
    f = O.fit(X, y, [0.5, 0.8], O.SE, 1.0, 0.01)
    K = O.gram(O.SE, X, [0.5, 0.8], 1.0, 0.01)
    a, b, c, d = K[0, 0], K[0, 1], K[1, 0], K[1, 1]
    det = a * d - b * c
    Kinv = np.array([[d, -b], [-c, a]]) / det
    yt = (y - y.mean()) / y.std()
    assert np.allclose(f.alpha, Kinv @ yt, rtol=1e-13, atol=1e-13)
    r = _rng(8)
    Xb = r.uniform(0, 1, (60, 4))
    yb = r.normal(size=60)
    fb = O.fit(Xb, yb, [0.5] * 4, O.MATERN52, 1.0, 1e-4)
    Kb = O.gram(O.MATERN52, Xb, [0.5] * 4, 1.0, 1e-4)
    ytb = (yb - yb.mean()) / yb.std()
    res = np.abs(Kb @ fb.alpha - ytb).max()
    assert res <= 1e-13 * np.linalg.cond(Kb) * np.abs(ytb).max()


def test_fit_rejects_empty():
    f = O.fit(np.zeros((0, 3)), np.zeros(0), [1.0] * 3)
    assert f.status == O.INVALID


def test_centre_only_option():
    r = _rng(9)
    X = r.uniform(0, 1, (10, 2))
    y = r.normal(size=10) * 5
    f = O.fit(X, y, [0.5, 0.5], O.SE, 1.0, 1e-3, normalize_y=False)
    assert f.ystd == 1.0
    f0 = O.fit(X, np.full(10, 3.0), [0.5, 0.5], O.SE, 1.0, 1e-3)
    assert f0.ystd == 1.0  # zero spread falls back to unit scale


# ---------------------------------------------------------------------------
# Posterior
# ---------------------------------------------------------------------------

def test_noise_free_interpolation():
    r = _rng(10)
    n = 12
    X = r.uniform(0, 1, (n, 2))
    y = r.normal(size=n) * 2 + 3
    for kind in (O.SE, O.MATERN52):
        f = O.fit(X, y, [0.25, 0.25], kind, 1.0, 0.0)
        assert f.status == O.OK
        s = O.score(f, X)
        assert np.abs(s["mu"] - y).max() <= 1e-10 * np.abs(y).max()
        assert (s["sigma"] ** 2).max() <= 1e-10


def test_posterior_n1_closed_form():
    x1 = np.array([[0.2, 0.7]])
    y = np.array([2.5])
    ls = [0.4, 0.9]
    sf2, sn2 = 1.3, 0.2
    f = O.fit(x1, y, ls, O.SE, sf2, sn2, normalize_y=False)
    xs = np.array([[0.5, 0.1], [0.2, 0.7]])
    s = O.score(f, xs)
    for j in range(2):
        k = O.kernel(O.SE, xs[j], x1[0], ls, sf2)
        # centred y_1 is zero: mean equals ymean, variance sf2 - k^2 / (sf2 + sn2)
        assert s["mu"][j] == pytest.approx(2.5, rel=1e-15)
        assert s["sigma"][j] == pytest.approx(math.sqrt(sf2 - k * k / (sf2 + sn2)), rel=1e-14)
    # two points, one of which is far: the n = 1 closed form for the mean
    X2 = np.array([[0.2, 0.7], [50.0, 50.0]])
    y2 = np.array([2.0, -1.0])
    f2 = O.fit(X2, y2, ls, O.SE, sf2, sn2, normalize_y=False)
    s2 = O.score(f2, xs[:1])
    k = O.kernel(O.SE, xs[0], X2[0], ls, sf2)
    mean = 0.5
    want = mean + k * (2.0 - mean) / (sf2 + sn2)
    assert s2["mu"][0] == pytest.approx(want, rel=1e-14)


def test_score_bound_n1_equals_posterior():
    """One observation: the nearest-observation bound is the posterior itself
    (the single-point conditional variance sf2 - k^2 / (sf2 + sn2))."""
    x1 = np.array([[0.2, 0.7]])
    f = O.fit(x1, np.array([2.5]), [0.4, 0.9], O.SE, 1.3, 0.2, normalize_y=False)
    xs = np.array([[0.5, 0.1], [0.2, 0.7], [0.9, 0.95]])
    s = O.score(f, xs)
    b = O.score_bound(f, xs)
    assert np.allclose(b["mu"], s["mu"], rtol=1e-15, atol=0)
    assert np.allclose(b["sigma_ub"], s["sigma"], rtol=1e-14, atol=0)
    assert np.allclose(b["ei_ub"], s["ei"], rtol=1e-13, atol=0)


def test_score_bound_n2_brute_force():
    """Two observations: the bound is the smaller of the two single-point
    conditional variances, written out by hand, and it is not below the
    two-point posterior variance."""
    X = np.array([[0.1, 0.3], [0.6, 0.4]])
    y = np.array([1.0, -0.5])
    ls, sf2, sn2 = [0.3, 0.5], 0.8, 0.05
    f = O.fit(X, y, ls, O.MATERN52, sf2, sn2)
    xs = np.array([[0.2, 0.3], [0.5, 0.5], [0.35, 0.35]])
    b = O.score_bound(f, xs)
    s = O.score(f, xs)
    for j in range(3):
        k = [O.kernel(O.MATERN52, xs[j], X[i], ls, sf2) for i in range(2)]
        v1 = [sf2 - ki * ki / (sf2 + sn2) for ki in k]
        want = f.ystd * math.sqrt(min(v1))
        assert b["sigma_ub"][j] == pytest.approx(want, rel=1e-14)
        assert b["sigma_ub"][j] >= s["sigma"][j]
        assert b["ei_ub"][j] == pytest.approx(O.ei(b["mu"][j], b["sigma_ub"][j], f.fbest), rel=1e-14)


def test_score_bound_dominates_posterior():
    r = _rng(21)
    X = r.uniform(0, 1, (40, 3))
    y = r.normal(size=40)
    f = O.fit(X, y, [0.3, 0.5, 0.4], O.SE, 1.2, 1e-3)
    Xc = r.uniform(0, 1, (300, 3))
    s = O.score(f, Xc)
    b = O.score_bound(f, Xc)
    assert np.allclose(b["mu"], s["mu"], rtol=1e-13, atol=1e-13)
    assert np.all(b["sigma_ub"] >= s["sigma"] * (1 - 1e-12))
    assert np.all(b["ei_ub"] >= s["ei"] * (1 - 1e-12) - 1e-15)
    assert np.any(b["sigma_ub"] > s["sigma"] * 1.01)  # a bound, not an identity


def test_posterior_far_field_is_prior():
    r = _rng(11)
    X = r.uniform(0, 1, (15, 3))
    y = r.normal(size=15) * 4 + 7
    f = O.fit(X, y, [0.2] * 3, O.SE, 1.5, 1e-3)
    s = O.score(f, np.full((2, 3), 100.0))
    assert np.allclose(s["mu"], y.mean(), rtol=1e-15)
    assert np.allclose(s["sigma"], y.std() * math.sqrt(1.5), rtol=1e-15)


def test_posterior_permutation_invariant_and_matches_library():
    r = _rng(12)
    n = 40
    X = r.uniform(0, 1, (n, 3))
    y = r.normal(size=n)
    Xc = r.uniform(0, 1, (30, 3))
    ls = [0.3, 0.5, 0.4]
    f = O.fit(X, y, ls, O.MATERN52, 1.0, 1e-3)
    s = O.score(f, Xc)
    perm = r.permutation(n)
    fp = O.fit(X[perm], y[perm], ls, O.MATERN52, 1.0, 1e-3)
    sp = O.score(fp, Xc)
    for k in ("mu", "sigma", "ei"):
        assert np.allclose(s[k], sp[k], rtol=1e-10, atol=1e-12)
    # library special case: posterior through numpy.linalg.solve on K
    K = O.gram(O.MATERN52, X, ls, 1.0, 1e-3)
    Ks = np.array([[O.kernel(O.MATERN52, a, b, ls) for b in X] for a in Xc])
    yt = (y - y.mean()) / y.std()
    mu = y.mean() + y.std() * Ks @ np.linalg.solve(K, yt)
    var = 1.0 - np.einsum("ij,ji->i", Ks, np.linalg.solve(K, Ks.T))
    assert np.allclose(s["mu"], mu, rtol=1e-10)
    assert np.allclose(s["sigma"], y.std() * np.sqrt(var), rtol=1e-8)


# ---------------------------------------------------------------------------
# Expected improvement
# ---------------------------------------------------------------------------

def test_ei_golden_normal_table():
    g = _golden("normal_values.json")
    for p in g["points"]:
        z = p["z"]
        sigma = 1.7
        mu = 3.0
        f = mu + z * sigma
        want = sigma * (z * p["Phi"] + p["phi"])
        assert O.ei(mu, sigma, f) == pytest.approx(want, rel=1e-13)
        # improvement below the incumbent is still positive (exploration term)
        f2 = mu - z * sigma
        want2 = sigma * (-z * (1 - p["Phi"]) + p["phi"])
        assert O.ei(mu, sigma, f2) == pytest.approx(want2, rel=1e-11)


def test_ei_special_cases_and_monotonicity():
    assert O.ei(2.0, 0.5, 2.0) == pytest.approx(0.5 / math.sqrt(2 * math.pi), rel=1e-15)
    assert O.ei(1.0, 0.0, 3.0) == 2.0
    assert O.ei(4.0, 0.0, 3.0) == 0.0
    assert O.ei(1.0, 1e-300, 3.0) == pytest.approx(2.0, rel=1e-15)
    mus = np.linspace(-3, 3, 41)
    v = [O.ei(m, 0.8, 0.0) for m in mus]
    assert all(a > b for a, b in zip(v, v[1:]))
    sig = np.linspace(0.01, 4, 41)
    w = [O.ei(0.5, s, 0.0) for s in sig]
    assert all(a < b for a, b in zip(w, w[1:]))


def test_ei_against_scipy_norm():
    r = _rng(13)
    for _ in range(50):
        mu, sigma, f = r.normal(), r.uniform(0.01, 3), r.normal()
        z = (f - mu) / sigma
        want = (f - mu) * scipy.stats.norm.cdf(z) + sigma * scipy.stats.norm.pdf(z)
        # the two closed-form terms cancel for z << 0, so far in the lower
        # tail only an absolute bound on the scale of sigma is meaningful
        tol = 1e-12 * want if z > -6 else 1e-15 * sigma
        assert abs(O.ei(mu, sigma, f) - want) <= tol


@pytest.mark.slow
def test_ei_monte_carlo():
    r = _rng(14)
    for mu, sigma, f in [(0.3, 1.1, 0.0), (-1.0, 0.4, -0.8), (2.0, 2.0, 0.5)]:
        F = r.normal(mu, sigma, size=10_000_000)
        imp = np.maximum(f - F, 0.0)
        est = imp.mean()
        se = imp.std() / math.sqrt(imp.size)
        assert abs(O.ei(mu, sigma, f) - est) <= 5 * se


# ---------------------------------------------------------------------------
# Argmax and top-k
# ---------------------------------------------------------------------------

def test_argmax_and_topk_brute_force():
    r = _rng(15)
    v = np.round(r.normal(size=500), 1)  # many exact ties
    order = sorted(range(500), key=lambda j: (-v[j], j))
    assert O.argmax(v) == order[0]
    assert list(O.topk(v, 37)) == order[:37]
    v2 = v.copy()
    v2[order[0]] = np.nan
    assert O.argmax(v2) == order[1]
    # exact tie at the maximum: the lowest index wins
    v3 = np.zeros(10)
    v3[[3, 6, 8]] = 2.0
    assert O.argmax(v3) == 3
    assert list(O.topk(v3, 4)) == [3, 6, 8, 0]


# ---------------------------------------------------------------------------
# Synthetic objective (input generator) pins
# ---------------------------------------------------------------------------

def test_synthetic_hand_values():
    g = _golden("synthetic_values.json")
    specs = {"c1": I.spec_c1(), "c2": I.spec_grouped(20, 0.1), "c5": I.spec_grouped(40, 0.2)}
    for name, spec in specs.items():
        d = g[name]["d"]
        assert I.synthetic_f(np.zeros(d), spec) == pytest.approx(g[name]["f0"], abs=1e-12)
        assert I.synthetic_f(np.ones(d), spec) == pytest.approx(g[name]["f1"], abs=1e-12)
        if "fhalf" in g[name]:
            assert I.synthetic_f(np.full(d, 0.5), spec) == pytest.approx(g[name]["fhalf"], abs=1e-12)


def _mixed_difference(f, x, i, j, h=0.05):
    ei = np.zeros_like(x)
    ej = np.zeros_like(x)
    ei[i] = h
    ej[j] = h
    return f(x + ei + ej) - f(x + ei) - f(x + ej) + f(x)


def test_separability_zero_interaction_without_coupling():
    """Independent routines: with no cross-group coupling, the mixed difference
    across groups vanishes up to summation rounding (mirrors the paper's
    finding that the independent groups show no external influence,
    Sec. IV-C)."""
    r = _rng(16)
    spec0 = I.spec_grouped(20, 0.0)
    f0 = lambda x: I.synthetic_f(x, spec0)
    for _ in range(20):
        x = r.uniform(0, 0.9, 20)
        i, j = 2, 7
        val = f0(x)
        assert abs(_mixed_difference(f0, x, i, j)) <= 8 * np.spacing(abs(val)) * 4
    # with coupling the first variables of adjacent groups interact, growing with lambda
    x = r.uniform(0, 0.9, 20)
    ints = []
    for lam in (0.1, 0.5, 1.0):
        spec = I.spec_grouped(20, lam)
        ints.append(abs(_mixed_difference(lambda z: I.synthetic_f(z, spec), x, 0, 5)))
    assert ints[0] > 1e-6 and ints[0] < ints[1] < ints[2]
    # within a group the pair term always couples
    assert abs(_mixed_difference(f0, x, 0, 1)) > 1e-4


def test_inputs_float32_representable_and_seeded():
    p = I.make_config("c2-s", n=64, m=256)
    assert np.array_equal(p.X, p.X.astype(np.float32).astype(np.float64))
    assert np.array_equal(p.Xc, p.Xc.astype(np.float32).astype(np.float64))
    q = I.make_config("c2-s", n=64, m=256)
    assert np.array_equal(p.X, q.X) and np.array_equal(p.y, q.y)
    assert np.allclose(p.lengthscale / math.sqrt(20),
                       I.make_config("c2", n=64, m=256).lengthscale)


# ---------------------------------------------------------------------------
# MLP ensemble
# ---------------------------------------------------------------------------

def _small_mlp(seed=0, E=2, D=3, H=5):
    r = _rng(seed)
    init = I.mlp_init(r, members=E, d_in=D, hidden=H)
    return O.mlp_pack(**init), D, H


def test_gelu_against_normal_cdf():
    for u in (-3.0, -0.7, 0.0, 0.4, 2.5):
        assert O.gelu(u) == pytest.approx(u * scipy.stats.norm.cdf(u), rel=1e-14, abs=1e-300)
        h = 1e-6
        fd = (u + h) * scipy.stats.norm.cdf(u + h) - (u - h) * scipy.stats.norm.cdf(u - h)
        assert O.gelu_grad(u) == pytest.approx(fd / (2 * h), rel=1e-8)


def test_bf16_rounding_matches_torch():
    import torch
    r = _rng(17)
    vals = np.concatenate([r.normal(size=2000) * 10.0 ** r.integers(-8, 8, 2000),
                           [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38]])
    t = torch.tensor(vals, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64)
    ours = np.array([O.bf16(v) for v in vals])
    assert np.array_equal(ours, t.numpy())


def test_mlp_gradient_finite_differences():
    params, D, H = _small_mlp(1)
    r = _rng(2)
    X = r.uniform(0, 1, (7, D))
    yt = r.normal(size=7)
    loss, g = O.mlp_loss_grad(params, D, H, X, yt)
    h = 1e-6
    for e in range(params.shape[0]):
        for k in range(params.shape[1]):
            p1 = params.copy()
            p2 = params.copy()
            p1[e, k] += h
            p2[e, k] -= h
            l1, _ = O.mlp_loss_grad(p1, D, H, X, yt)
            l2, _ = O.mlp_loss_grad(p2, D, H, X, yt)
            fd = (l1[e] - l2[e]) / (2 * h)
            assert abs(fd - g[e, k]) <= 1e-6 * max(abs(g[e, k]), 1e-3)


def test_mlp_forward_matches_direct_formula():
    params, D, H = _small_mlp(3)
    r = _rng(4)
    X = r.uniform(0, 1, (6, D))
    out = O.mlp_forward(params, D, H, X)
    gelu = lambda u: u * scipy.stats.norm.cdf(u)
    for e in range(params.shape[0]):
        p = params[e]
        W1 = p[:H * D].reshape(H, D)
        b1 = p[H * D:H * D + H]
        o = H * D + H
        W2 = p[o:o + H * H].reshape(H, H)
        b2 = p[o + H * H:o + H * H + H]
        w3 = p[o + H * H + H:o + H * H + 2 * H]
        b3 = p[-1]
        ref = gelu(gelu(X @ W1.T + b1) @ W2.T + b2) @ w3 + b3
        assert np.allclose(out[e], ref, rtol=1e-12, atol=1e-13)


def test_mlp_bf16_emulation_is_close_but_distinct():
    params, D, H = _small_mlp(5, E=1, D=20, H=64)
    X = _rng(6).uniform(0, 1, (32, 20))
    a = O.mlp_forward(params, 20, 64, X)
    b = O.mlp_forward(params, 20, 64, X, bf16=True)
    assert not np.array_equal(a, b)
    assert np.abs(a - b).max() < 0.05 * np.abs(a).max() + 0.02


def test_adam_first_step_closed_form():
    r = _rng(7)
    w0 = r.normal(size=50)
    g = r.normal(size=50)
    w = w0.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    O.adam_step(w, m, v, g, 1, lr=1e-3)
    assert np.allclose(w - w0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    # second step against a hand-unrolled update
    g2 = r.normal(size=50)
    mm = 0.9 * (0.1 * g) + 0.1 * g2
    vv = 0.999 * (0.001 * g * g) + 0.001 * g2 * g2
    want = w - 1e-3 * (mm / (1 - 0.81)) / (np.sqrt(vv / (1 - 0.999 ** 2)) + 1e-8)
    O.adam_step(w, m, v, g2, 2, lr=1e-3)
    assert np.allclose(w, want, rtol=1e-12, atol=1e-15)


def test_mlp_training_reduces_loss():
    params, D, H = _small_mlp(8, E=2, D=4, H=16)
    r = _rng(9)
    X = r.uniform(0, 1, (64, 4))
    yt = np.sin(3 * X[:, 0]) + X[:, 1] ** 2
    yt = (yt - yt.mean()) / yt.std()
    _, hist = O.mlp_train(params, D, H, X, yt, steps=100, lr=1e-2)
    assert np.all(hist[-1] < 0.5 * hist[0])
    assert np.all(np.diff(hist[:20], axis=0) < 0)


def test_ensemble_ei_against_numpy():
    r = _rng(18)
    out = r.normal(size=(5, 40))
    mu, sd, e = O.ens_ei(out, -0.2)
    assert np.allclose(mu, out.mean(0), rtol=1e-14)
    assert np.allclose(sd, out.std(0), rtol=1e-13)
    for i in range(40):
        z = (-0.2 - mu[i]) / sd[i]
        want = (-0.2 - mu[i]) * scipy.stats.norm.cdf(z) + sd[i] * scipy.stats.norm.pdf(z)
        assert e[i] == pytest.approx(want, rel=1e-11)


def test_ensemble_lcb_special_cases():
    """kappa = 0 ranks by the negated mean; two members a -/+ delta give
    -(a - kappa delta); a single member has zero spread."""
    a = np.array([0.3, -1.2, 2.0])
    dl = np.array([0.1, 0.5, 0.0])
    out = np.stack([a - dl, a + dl])
    assert np.allclose(O.ens_lcb(out, 0.0), -a, rtol=0, atol=1e-15)
    assert np.allclose(O.ens_lcb(out, 2.0), -(a - 2.0 * dl), rtol=0, atol=1e-15)
    assert np.allclose(O.ens_lcb(a[None, :], 3.0), -a, rtol=0, atol=1e-15)
