"""GPU parity of the hyperparameter fitting (gpbo_lml_grad_batched,
gpbo_fit_hyper_batched) against the float64 oracle, through the C ABI.

Bars:
* gradient: |g - g_oracle| <= 64 n eps cond(K) (1 + max |g_oracle|) per
  entry (K^-1 from the inverse factor carries the forward error of the
  factorisation, eps cond(K) relative), LML to the fit's own bar;
* optimiser, first steps (large gradients, Adam's normalised steps move
  theta by ~lr): the winning start's theta within 1e-7 and its LML within
  1e-9 (relative) of the oracle's;
* optimiser, long run: the final LML within 1e-3 (relative, + 1e-3) of the
  oracle's optimum (near the optimum Adam's steps depend on the sign of
  near-zero gradients, so the paths may part at the lr scale), the reported
  LML equal to the oracle's LML at the returned theta (1e-9), and the
  returned model fitted at that theta;
* jitter: a singular K takes the same jitter as the oracle's policy.
"""
import math

import numpy as np
import pytest
import torch

from oracle import hyper as OH
from oracle import oracle as O
from paper_2403_08131_amd import gpbo as G

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx():
    c = G.Context(0)
    yield c
    c.close()


def _t(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def _okind(k):
    return O.SE if k == G.KERNEL_SE else O.MATERN52


def _data(n, d, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(size=(n, d))
    y = np.sin(5.0 * X[:, 0]) + np.sum(X[:, 1:] ** 2, axis=1) + 0.05 * rng.standard_normal(n)
    return X, y


CASES = [(5, 2, G.KERNEL_SE, True), (64, 3, G.KERNEL_MATERN52, True),
         (100, 4, G.KERNEL_SE, False), (300, 6, G.KERNEL_MATERN52, True),
         (700, 5, G.KERNEL_SE, True)]


def test_lml_grad_matches_oracle(ctx):
    models, refs = [], []
    for i, (n, d, kind, norm) in enumerate(CASES):
        X, y = _data(n, d, 60 + i)
        ls = 0.3 + 0.1 * np.arange(d)
        sf2, sn2 = 1.2, 1e-2
        models.append(G.fit(ctx, _t(X), _t(y), list(ls), kind, sf2, sn2, normalize_y=norm))
        st, g, l = O.lml_grad(X, y, ls, _okind(kind), sf2, sn2, norm)
        assert st == O.OK
        cond = np.linalg.cond(O.gram(_okind(kind), X, ls, sf2, sn2))
        refs.append((g, l, cond, n))
    print("lml grad parity", [c[:2] for c in CASES], flush=True)
    grad, lml = G.lml_grad_batched(ctx, models)
    grad, lml = grad.cpu().numpy(), lml.cpu().numpy()
    for b, (g, l, cond, n) in enumerate(refs):
        d = CASES[b][1]
        tol = 64 * n * EPS * cond * (1.0 + np.max(np.abs(g)))
        err = np.max(np.abs(grad[b, :d + 2] - g))
        assert err <= tol, (b, err, tol)
        assert np.all(grad[b, d + 2:] == 0.0)
        assert lml[b] == pytest.approx(l, rel=64 * n * EPS * cond, abs=64 * n * EPS * cond * n)
    for mo in models:
        mo.free()


def test_lml_grad_of_failed_fit_is_nan(ctx):
    x = np.array([[0.25, 0.75], [0.25, 0.75]])
    m = G.fit_async(ctx, _t(x), _t([1.0, 2.0]), [0.5, 0.5], G.KERNEL_SE, 1.0, 0.0)
    grad, lml = G.lml_grad_batched(ctx, [m])
    assert np.all(np.isnan(grad.cpu().numpy())) and np.isnan(lml.item())
    with pytest.raises(G.GpboError):
        m.status()
    m.free()


def _starts(rng, S, d):
    th = np.empty((S, d + 2))
    th[:, :d] = np.log(rng.uniform(0.1, 1.0, size=(S, d)))
    th[:, d] = np.log(rng.uniform(0.5, 2.0, size=S))
    th[:, d + 1] = np.log(rng.uniform(1e-4, 1e-1, size=S))
    return th


def _bounds(d):
    lo = np.concatenate([np.full(d, math.log(1e-2)), [math.log(1e-2), math.log(1e-6)]])
    hi = np.concatenate([np.full(d, math.log(1e2)), [math.log(1e2), math.log(1.0)]])
    return lo, hi


@pytest.mark.parametrize("steps", [6, 150])
def test_fit_hyper_matches_oracle(ctx, steps):
    specs = [(30, 2, G.KERNEL_SE), (80, 3, G.KERNEL_MATERN52)]
    S = 3
    rng = np.random.default_rng(5 + steps)
    data = [_data(n, d, 90 + n) for n, d, _ in specs]
    ldt = max(d for _, d, _ in specs) + 2
    th0 = np.zeros((len(specs), S, ldt))
    lo = np.zeros((len(specs), ldt))
    hi = np.zeros((len(specs), ldt))
    for b, (n, d, _) in enumerate(specs):
        th0[b, :, :d + 2] = _starts(rng, S, d)
        lo[b, :d + 2], hi[b, :d + 2] = _bounds(d)
    probs = [dict(X=_t(X), y=_t(y), kernel=kind) for (X, y), (_, _, kind) in zip(data, specs)]
    print(f"fit_hyper steps={steps}", flush=True)
    st, status, th, lml, jit, models = G.fit_hyper_batched(ctx, probs, th0, lo, hi, steps=steps,
                                                           lr=0.05)
    assert st == G.OK, status
    for b, ((X, y), (n, d, kind)) in enumerate(zip(data, specs)):
        best, res = OH.fit(X, y, th0[b, :, :d + 2], lo[b, :d + 2], hi[b, :d + 2], _okind(kind),
                           steps=steps, lr=0.05)
        ref = res[best]
        got = th[b, :d + 2]
        at_got = OH.lml_grad_jitter(X, y, got, _okind(kind))
        assert lml[b] == pytest.approx(at_got[2], rel=1e-9)
        assert jit[b] == 0.0 and ref["jitter"] == 0.0
        if steps <= 10:
            np.testing.assert_allclose(got, ref["theta"], rtol=0, atol=1e-7)
            assert lml[b] == pytest.approx(ref["lml"], rel=1e-9)
        else:
            assert lml[b] >= ref["lml"] - (1e-3 * abs(ref["lml"]) + 1e-3), (lml[b], ref["lml"])
        assert models[b].stats()["lml"] == pytest.approx(lml[b], rel=1e-9)
        models[b].free()


def test_fit_hyper_singular_kernel_matrix_takes_jitter(ctx):
    """Two identical points, SE, signal_var exactly 1, noise held at 1e-30:
    K's 2 x 2 block is [[1, 1], [1, 1]] in float64, the second pivot is
    exactly zero on any factorisation order, and the first jitter (1e-8)
    makes it positive.  (After steps move signal_var off 1 the pivot is a
    rounding residue whose sign depends on the order of operations, so the
    policy is compared at the start: zero steps, the final evaluation only.)"""
    X = np.array([[0.2, 0.4], [0.2, 0.4], [0.9, 0.1], [0.5, 0.5]])
    y = np.array([0.0, 0.1, 1.0, 0.4])
    th0 = np.log([[[0.3, 0.3, 1.0, 1e-30]]])
    lo = np.log([[1e-2, 1e-2, 1e-2, 1e-30]])
    hi = np.log([[1e2, 1e2, 1e2, 1e-30]])  # the noise is held at 1e-30
    st, status, th, lml, jit, models = G.fit_hyper_batched(ctx, [dict(X=_t(X), y=_t(y))], th0, lo,
                                                           hi, steps=0, lr=0.05)
    assert st == G.OK, status
    best, res = OH.fit(X, y, th0[0], lo[0], hi[0], O.SE, steps=0, lr=0.05)
    assert jit[0] == res[best]["jitter"] == 1e-8
    np.testing.assert_allclose(th[0], res[best]["theta"], rtol=0, atol=1e-7)
    cond = np.linalg.cond(O.gram(O.SE, X, [0.3, 0.3], 1.0, math.exp(th0[0, 0, 3]) + 1e-8))
    assert lml[0] == pytest.approx(res[best]["lml"], rel=64 * 4 * EPS * cond)
    models[0].free()
