"""Bayesian-optimisation driver for a set of independent tuning searches.

The loop of the paper's Sec. III-A -- fit the surrogate to the evaluated
configurations, let the acquisition function choose the next configuration,
evaluate it, retrain -- run for every search of a plan at once, with the
initial design and budget of Sec. IV-D (5 random configurations, 10
evaluations per tuned parameter).  Every arithmetic step runs in the
library: one batched fit at the start, then per iteration one batched
scoring call (expected improvement and its argmax for every active search)
and one batched rank-one update of the fitted models (gpbo_append_batched:
O(n^2) per search instead of a refit).  This module only carries the chosen
configurations to the objective and its values back, because the objective
is the application being tuned.

The candidate pool of each iteration is drawn uniformly over the search's
box by default; callers that need reproducible pools (the tests) pass their
own.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import gpbo as G


@dataclass
class Search:
    """One tuning search: the parameters it tunes (indices into the full
    configuration), their box and the surrogate's fixed hyperparameters."""
    dims: list
    lo: np.ndarray
    hi: np.ndarray
    lengthscale: np.ndarray
    kernel: int = G.KERNEL_SE
    signal_var: float = 1.0
    noise_var: float = 1e-4
    normalize_y: bool = True

    @property
    def d(self):
        return len(self.dims)


@dataclass
class Result:
    """History of one search: all evaluations in order (initial design
    first), the pool index chosen at each iteration and the winning EI."""
    X: np.ndarray
    y: np.ndarray
    picks: list = field(default_factory=list)
    ei_max: list = field(default_factory=list)

    @property
    def best(self):
        i = int(np.argmin(self.y))
        return self.X[i], float(self.y[i])


def _uniform_pool(gen, m, s: Search, device, dtype):
    lo = torch.as_tensor(np.asarray(s.lo), dtype=dtype, device=device)
    hi = torch.as_tensor(np.asarray(s.hi), dtype=dtype, device=device)
    u = torch.rand((m, s.d), generator=gen, dtype=dtype, device=device)
    return lo + (hi - lo) * u


def run(ctx: G.Context, searches, evaluate, n_init=5, evals_per_dim=10, pool_size=4096,
        prec="fp64", init=None, pools=None, seed=0, update="append"):
    """Run every search to its budget.

    evaluate(b, X) -> values: the objective of search b at the rows of X
      (host float64, k x d_b); returns k float64 values (lower is better).
    init: optional list of host arrays (n_init x d_b), the initial designs
      (default: uniform in the box from a generator seeded with ``seed``).
    pools(t, b) -> device tensor (m x d_b): optional candidate pool of search
      b at iteration t, float64 for prec "fp64" else float32 (default:
      ``pool_size`` uniform candidates).
    update: "append" (rank-one update of the fitted models) or "refit" (a
      batched fit on all observations every iteration; for comparison).
    Returns a list of :class:`Result`, one per search."""
    dev = ctx.device
    B = len(searches)
    pdt = torch.float64 if prec == "fp64" else torch.float32
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    res, Xd, yd = [], [], []
    for b, s in enumerate(searches):
        X0 = (np.asarray(init[b], dtype=np.float64) if init is not None else
              _uniform_pool(gen, n_init, s, dev, torch.float64).cpu().numpy())
        y0 = np.asarray(evaluate(b, X0), dtype=np.float64)
        res.append(Result(X0.copy(), y0.copy()))
        Xd.append(torch.as_tensor(X0, device=dev).contiguous())
        yd.append(torch.as_tensor(y0, device=dev).contiguous())
    probs = [dict(X=Xd[b], y=yd[b], lengthscale=list(s.lengthscale), kernel=s.kernel,
                  signal_var=s.signal_var, noise_var=s.noise_var, normalize_y=s.normalize_y)
             for b, s in enumerate(searches)]
    st, models, status, _ = G.fit_batched(ctx, probs)
    if st != G.OK:
        raise G.GpboError(st, f"initial fit failed: statuses {status}")
    iters = [max(evals_per_dim * s.d - res[b].X.shape[0], 0) for b, s in enumerate(searches)]
    dmax = max(s.d for s in searches)
    # per iteration: scoring, the chosen rows and their read-back queued back
    # to back with one synchronisation; the values go up with the update
    stream = torch.cuda.current_stream(dev)
    xn = torch.zeros((B, dmax), dtype=torch.float64, device=dev)
    yd_new = torch.zeros(B, dtype=torch.float64, device=dev)
    xh = torch.empty((B, dmax), dtype=torch.float64, pin_memory=True)
    amh = torch.empty(B, dtype=torch.int64, pin_memory=True)
    emh = torch.empty(B, dtype=torch.float64, pin_memory=True)
    yh = torch.empty(B, dtype=torch.float64, pin_memory=True)
    try:
        for t in range(max(iters) if iters else 0):
            act = [b for b in range(B) if t < iters[b]]
            na = len(act)
            ma = [models[b] for b in act]
            P = [pools(t, b) if pools is not None else
                 _uniform_pool(gen, pool_size, searches[b], dev, pdt) for b in act]
            _, am, em = G.score_batched(ctx, ma, P, prec=prec, want=())
            G.next_batched(ctx, ma, P, prec, am, xn[:na])
            xh[:na].copy_(xn[:na], non_blocking=True)
            amh[:na].copy_(am, non_blocking=True)
            emh[:na].copy_(em, non_blocking=True)
            stream.synchronize()
            xv, amv, emv = xh.numpy(), amh.numpy(), emh.numpy()
            yv = yh.numpy()
            for k, b in enumerate(act):
                x = xv[k, :searches[b].d].copy()
                yv[k] = float(np.asarray(evaluate(b, x[None, :]), dtype=np.float64).reshape(-1)[0])
                r = res[b]
                r.X = np.vstack([r.X, x[None, :]])
                r.y = np.append(r.y, yv[k])
                r.picks.append(int(amv[k]))
                r.ei_max.append(float(emv[k]))
            if update == "append":
                # yh is rewritten only after the next iteration's synchronisation
                yd_new[:na].copy_(yh[:na], non_blocking=True)
                G.append_batched(ctx, ma, xn[:na], yd_new[:na])
            else:
                for b in act:
                    models[b].free()
                    probs[b]["X"] = torch.as_tensor(res[b].X, device=dev).contiguous()
                    probs[b]["y"] = torch.as_tensor(res[b].y, device=dev).contiguous()
                st, fresh, status, _ = G.fit_batched(ctx, [probs[b] for b in act])
                if st != G.OK:
                    raise G.GpboError(st, f"refit failed: statuses {status}")
                for k, b in enumerate(act):
                    models[b] = fresh[k]
        st, status, _ = G.status_batched(ctx, models)
        if st != G.OK:
            raise G.GpboError(st, f"rank-one update failed: statuses {status}")
    finally:
        for mo in models:
            if mo is not None:
                mo.free()
    return res
