"""Plain reference of the Bayesian-optimisation loop of one tuning search
(the paper's Sec. III-A and IV-D).  TEST INFRASTRUCTURE ONLY: the tests and
the benchmark's CPU legs import it; the product path never does, and it
shares no code with the library or its driver.

One search, with the surrogate's hyperparameters held fixed:

1. start from ``n_init`` evaluated configurations (Sec. IV-D starts every
   search from 5 random ones);
2. fit the Gaussian process to all evaluated configurations -- here from
   scratch every time, which is the definition a rank-one update of the
   fitted model has to reproduce (Sec. III-A calls this step re-training);
3. score the iteration's candidate pool by expected improvement against the
   best evaluation so far;
4. evaluate the objective at the pool's argmax (lowest index among equal
   values) and add the pair to the evaluated configurations;
5. repeat until the budget is spent (Sec. IV-D: 10 evaluations per tuned
   parameter, the initial ones included).

The candidate pools are inputs: the random numbers the loop draws come from
the seeded input module, so that a device run sees the same pools.

Parity status: pinned in tests/test_oracle_bo.py (each pick is the argmax of
an expected improvement computed by an independent dense-solve route, the
evaluated set grows by exactly the picked rows, the best value never rises,
and a one-dimensional case whose pool holds the objective's minimiser finds
it).
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def search(objective, X0, y0, pools, ls, kind=O.SE, sf2=1.0, sn2=1e-4, normalize_y=True):
    """Run one search.  ``objective(x)`` returns the value at one
    configuration (float64, shape (d,)); ``X0`` (n_init, d) and ``y0``
    (n_init,) are the initial evaluations; ``pools`` is a sequence of
    candidate arrays (m_t, d), one per iteration.

    Returns a dict: ``picks`` (pool index per iteration), ``X`` and ``y`` (all
    evaluations, initial ones first), ``ei_max`` (the winning EI per
    iteration), ``ei_gap`` (relative gap between the two largest EI values
    per iteration, for near-tie checks) and ``fbest`` (best value after each
    iteration)."""
    X = np.array(X0, dtype=np.float64, copy=True)
    y = np.array(y0, dtype=np.float64, copy=True)
    picks, ei_max, ei_gap, fbest = [], [], [], []
    for P in pools:
        P = np.asarray(P, dtype=np.float64)
        f = O.fit(X, y, ls, kind, sf2, sn2, normalize_y)
        if f.status != O.OK:
            raise RuntimeError(f"oracle fit failed at n={X.shape[0]} (pivot {f.bad_pivot})")
        ei = O.score(f, P, want=("ei",))["ei"]
        j = O.argmax(ei)
        top = np.sort(ei)[::-1]
        gap = (top[0] - top[1]) / max(abs(top[0]), 1e-300) if top.size > 1 else np.inf
        x = P[j].copy()
        X = np.vstack([X, x[None, :]])
        y = np.append(y, float(objective(x)))
        picks.append(j)
        ei_max.append(float(ei[j]))
        ei_gap.append(float(gap))
        fbest.append(float(y.min()))
    return {"picks": picks, "X": X, "y": y, "ei_max": ei_max, "ei_gap": ei_gap, "fbest": fbest}
