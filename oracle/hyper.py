"""Plain reference of the surrogate's hyperparameter fitting: maximise the
log marginal likelihood over theta = (log l_1 .. log l_d, log sf2, log sn2)
from several starting points.  TEST INFRASTRUCTURE ONLY: the tests and the
benchmark's CPU legs import it; the product path never does, and it shares
no code with the library.

The paper trains a Gaussian process on each search's evaluations (Sec.
IV-D) and does not say how its hyperparameters are chosen; this is the
usual choice, in these steps:

1. from each start theta_0 (inputs, like every random number here), take
   ``steps`` Adam steps (Kingma & Ba 2015, Alg. 1) up the gradient of the
   log marginal likelihood (Rasmussen & Williams 2006, eq. 5.9; the oracle's
   ``lml_grad``), each step clipped to the box [lo, hi];
2. a fit that fails (K not positive definite in floating point) is retried
   with jitter added to the noise variance: sf2 * jitter0 * 10^k for
   k = 0 .. retries - 1 (the gradient with respect to log sn2 stays that of
   sn2 itself); a start whose retries all fail is abandoned (LML -inf);
3. after the last step the LML at the final theta is evaluated the same
   way, and the start with the largest LML wins (lowest index among equal
   values).

Parity status: pinned in tests/test_oracle_hyper.py (each step is the Adam
update of the independently pinned gradient, the final LML is at least the
starting LML on well-posed data, the optimum is stationary by central
differences of the LML, data drawn from a Gaussian process with known
hyperparameters give them back within their sampling spread, and a
singular K takes the jitter path).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

JITTER0 = 1e-8
RETRIES = 4


def lml_grad_jitter(X, y, theta, kind, normalize_y=True, jitter0=JITTER0, retries=RETRIES):
    """(status, grad, lml, jitter): the gradient and LML at theta, with the
    jitter policy of step 2 (jitter = 0 when the plain fit succeeds)."""
    d = X.shape[1]
    ls = np.exp(theta[:d])
    sf2, sn2 = math.exp(theta[d]), math.exp(theta[d + 1])
    for k in range(retries + 1):
        jit = 0.0 if k == 0 else sf2 * jitter0 * 10.0 ** (k - 1)
        st, g, lml = O.lml_grad(X, y, ls, kind, sf2, sn2 + jit, normalize_y)
        if st == O.OK:
            g = g.copy()
            g[d + 1] *= sn2 / (sn2 + jit)  # derivative with respect to log sn2, not the jittered one
            return st, g, lml, jit
    return st, None, -math.inf, math.nan


def fit_start(X, y, theta0, lo, hi, kind=O.SE, steps=100, lr=0.05, normalize_y=True,
              beta1=0.9, beta2=0.999, eps=1e-8):
    """One start: returns dict(theta, lml, jitter, alive, lml0, path) where
    path holds theta after every step."""
    th = np.clip(np.asarray(theta0, dtype=np.float64), lo, hi)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    path = []
    lml0 = None
    for t in range(1, steps + 1):
        st, g, lml, _ = lml_grad_jitter(X, y, th, kind, normalize_y)
        if st != O.OK:
            return {"theta": th, "lml": -math.inf, "jitter": math.nan, "alive": False,
                    "lml0": lml0 if lml0 is not None else -math.inf, "path": path}
        if lml0 is None:
            lml0 = lml
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        th = np.clip(th + lr * mh / (np.sqrt(vh) + eps), lo, hi)
        path.append(th.copy())
    st, _, lml, jit = lml_grad_jitter(X, y, th, kind, normalize_y)
    if lml0 is None:
        lml0 = lml
    return {"theta": th, "lml": lml, "jitter": jit, "alive": st == O.OK, "lml0": lml0,
            "path": path}


def fit(X, y, starts, lo, hi, kind=O.SE, steps=100, lr=0.05, normalize_y=True):
    """All starts (rows of ``starts``); returns (best index, list of
    per-start results)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    res = [fit_start(X, y, s, lo, hi, kind, steps, lr, normalize_y) for s in np.asarray(starts)]
    best = 0
    for i, r in enumerate(res):
        if r["lml"] > res[best]["lml"]:
            best = i
    return best, res
