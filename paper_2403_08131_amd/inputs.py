"""Seeded synthetic inputs for the GP-fit / EI-scoring path.

This module is shared by the tests, the benchmark and the oracle driver.  It
draws random numbers and evaluates the synthetic objective, and holds none of
the Gaussian-process arithmetic: no kernel function, no factorisation, no
posterior, no acquisition.

Workloads (the paper's own objective needs an application that is not
available; these synthetic functions of controlled interdependence stand in
for the routines being tuned, Sec. III-C and Sec. IV-D of the paper):

* ``c1``  d=6, two disjoint groups of 3, f = sum cos(3 pi x)+x^2 plus the
  coupling 0.5 cos(pi (x0 - x3)); n=64 uniform observations, 4096 uniform
  candidates; Matern-5/2, lengthscale 0.2, signal variance 1, noise 1e-4.
* ``c2``  d=20, four groups of 5 with within-group pair coupling 0.3 x_i x_j
  and cross-group chain coupling lambda=0.1; n=512 scrambled-Sobol
  observations, 65536 candidates; SE-ARD, lengthscales log-uniform in
  [0.05, 1].
* ``c3``  64 independent sub-searches, d in {2..12}, n in [16, 400], 8192
  candidates each, two groups per problem, one lambda per batch.
* ``c4``  d=20 function as c2, 4096 uniform evaluations, a pool of
  1,048,576 candidates, MLP ensemble initial weights.
* ``c5``  d=40, eight groups of 5, lambda=0.2, n=2048, 262144 candidates.

The ``scaled`` variant multiplies every lengthscale by sqrt(d).  With the
literal lengthscales at d >= 20 the cross-covariances of almost every
candidate underflow (the posterior collapses to the prior), so correctness is
checked on the scaled variant while throughput is the same for both.

Observation noise is N(0, 0.01^2).  Observation and candidate coordinates are
rounded to float32-representable values at generation, so that a float32
kernel sees exactly the points the float64 oracle sees.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 240308131
NOISE_STD = 0.01
NOISE_VAR = 1e-4

KERNEL_SE = 0
KERNEL_MATERN52 = 1

CONFIG_IDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}


@dataclass
class SyntheticSpec:
    """Groups of coordinates and coupling constants of one synthetic objective."""
    groups: list            # list of lists of coordinate indices
    pair_coef: float        # within-group coefficient of x_i x_j over all pairs i<j
    lam: float              # cross-group chain coupling on each group's first variable


@dataclass
class Problem:
    """One sub-search: observations, candidate pool and fixed hyperparameters."""
    name: str
    d: int
    X: np.ndarray           # (n, d) float64, float32-representable
    y: np.ndarray           # (n,) float64
    Xc: np.ndarray          # (m, d) float64, float32-representable
    lengthscale: np.ndarray  # (d,) float64
    signal_var: float = 1.0
    noise_var: float = NOISE_VAR
    kernel: int = KERNEL_SE
    spec: SyntheticSpec = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def m(self):
        return self.Xc.shape[0]


def contiguous_groups(d, size):
    return [list(range(s, min(s + size, d))) for s in range(0, d, size)]


def synthetic_f(X, spec: SyntheticSpec):
    """Noise-free synthetic objective, evaluated row-wise on X (..., d).

    f(x) = sum_g [ sum_{i in G_g} (cos(3 pi x_i) + x_i^2)
                   + pair_coef * sum_{i<j in G_g} x_i x_j ]
           + lam * sum_{g=0}^{G-2} cos(pi (x_first(g) - x_first(g+1)))
    """
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros(X.shape[:-1], dtype=np.float64)
    for g in spec.groups:
        xs = X[..., g]
        out += np.sum(np.cos(3.0 * math.pi * xs) + xs * xs, axis=-1)
        if spec.pair_coef != 0.0:
            k = len(g)
            for a in range(k):
                for b in range(a + 1, k):
                    out += spec.pair_coef * xs[..., a] * xs[..., b]
    if spec.lam != 0.0:
        for gi in range(len(spec.groups) - 1):
            a = spec.groups[gi][0]
            b = spec.groups[gi + 1][0]
            out += spec.lam * np.cos(math.pi * (X[..., a] - X[..., b]))
    return out


def f32r(a):
    """Round to the nearest float32 and return float64 (exactly representable)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def _streams(config_id, replicate, n_streams=6):
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(config_id, replicate))
    return [np.random.default_rng(s) for s in ss.spawn(n_streams)]


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


def _sobol(rng, d, n):
    from scipy.stats import qmc
    seed = int(rng.integers(0, 2**31 - 1))
    eng = qmc.Sobol(d=d, scramble=True, seed=seed)
    m = int(round(math.log2(n)))
    if 2**m == n:
        return eng.random_base2(m)
    return eng.random(n)


def _observe(rng_noise, X, spec, noise=True):
    f = synthetic_f(X, spec)
    if noise:
        f = f + rng_noise.normal(0.0, NOISE_STD, size=f.shape)
    return f


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def spec_c1():
    return SyntheticSpec(groups=[[0, 1, 2], [3, 4, 5]], pair_coef=0.0, lam=0.5)


def spec_grouped(d, lam, size=5):
    return SyntheticSpec(groups=contiguous_groups(d, size), pair_coef=0.3, lam=lam)


def spec_two_groups(d, lam):
    h = (d + 1) // 2
    groups = [list(range(0, h))]
    if d - h > 0:
        groups.append(list(range(h, d)))
    return SyntheticSpec(groups=groups, pair_coef=0.3, lam=lam)


def make_c1(replicate=0, n=64, m=4096):
    r_ls, r_x, r_noise, r_c, _, _ = _streams(1, replicate)
    d = 6
    spec = spec_c1()
    X = f32r(r_x.uniform(0.0, 1.0, size=(n, d)))
    y = _observe(r_noise, X, spec)
    Xc = f32r(r_c.uniform(0.0, 1.0, size=(m, d)))
    return Problem("c1", d, X, y, Xc, np.full(d, 0.2), 1.0, NOISE_VAR,
                   KERNEL_MATERN52, spec)


def make_c2(replicate=0, scaled=False, n=512, m=65536, d=20, lam=0.1):
    r_ls, r_x, r_noise, r_c, _, _ = _streams(2, replicate)
    spec = spec_grouped(d, lam)
    ls = _log_uniform(r_ls, 0.05, 1.0, d)
    if scaled:
        ls = ls * math.sqrt(d)
    X = f32r(_sobol(r_x, d, n))
    y = _observe(r_noise, X, spec)
    Xc = f32r(r_c.uniform(0.0, 1.0, size=(m, d)))
    return Problem("c2-s" if scaled else "c2", d, X, y, Xc, ls, 1.0, NOISE_VAR,
                   KERNEL_SE, spec)


def make_c5(replicate=0, scaled=False, n=2048, m=262144, d=40, lam=0.2):
    r_ls, r_x, r_noise, r_c, _, _ = _streams(5, replicate)
    spec = spec_grouped(d, lam)
    ls = _log_uniform(r_ls, 0.05, 1.0, d)
    if scaled:
        ls = ls * math.sqrt(d)
    X = f32r(r_x.uniform(0.0, 1.0, size=(n, d)))
    y = _observe(r_noise, X, spec)
    Xc = f32r(r_c.uniform(0.0, 1.0, size=(m, d)))
    return Problem("c5-s" if scaled else "c5", d, X, y, Xc, ls, 1.0, NOISE_VAR,
                   KERNEL_SE, spec)


def make_c3(lam=0.1, replicate=0, scaled=False, B=64, m=8192,
            d_range=(2, 12), n_range=(16, 400)):
    """One batched launch of B independent sub-searches sharing one lambda."""
    lam_key = {0.0: 0, 0.1: 1, 0.5: 2}.get(float(lam), 3)
    r_shape, r_ls, r_x, r_noise, r_c, _ = _streams(3, replicate * 16 + lam_key)
    ds = r_shape.integers(d_range[0], d_range[1] + 1, size=B)
    ns = r_shape.integers(n_range[0], n_range[1] + 1, size=B)
    probs = []
    for b in range(B):
        d = int(ds[b])
        n = int(ns[b])
        spec = spec_two_groups(d, lam)
        ls = _log_uniform(r_ls, 0.05, 1.0, d)
        if scaled:
            ls = ls * math.sqrt(d)
        X = f32r(r_x.uniform(0.0, 1.0, size=(n, d)))
        y = _observe(r_noise, X, spec)
        Xc = f32r(r_c.uniform(0.0, 1.0, size=(m, d)))
        probs.append(Problem(f"c3[{b}]", d, X, y, Xc, ls, 1.0, NOISE_VAR,
                             KERNEL_SE, spec))
    return probs


def make_c4(replicate=0, n=4096, m=1048576, d=20, lam=0.1):
    """Learned-prescreen workload: GP observations, big pool, MLP initial weights.

    The GP uses the scaled lengthscales (sqrt(d) times log-uniform [0.05, 1]).
    """
    r_ls, r_x, r_noise, r_c, r_init, _ = _streams(4, replicate)
    spec = spec_grouped(d, lam)
    ls = _log_uniform(r_ls, 0.05, 1.0, d) * math.sqrt(d)
    X = f32r(r_x.uniform(0.0, 1.0, size=(n, d)))
    y = _observe(r_noise, X, spec)
    Xc = f32r(r_c.uniform(0.0, 1.0, size=(m, d)))
    p = Problem("c4", d, X, y, Xc, ls, 1.0, NOISE_VAR, KERNEL_SE, spec)
    p.extra["init_rng"] = r_init
    return p


def mlp_init(rng, members=5, d_in=20, hidden=256):
    """Initial MLP-ensemble weights, U(+-1/sqrt(fan_in)) for weights and biases.

    Returns float32 arrays shaped per member:
      W1 (E, H, d_in), b1 (E, H), W2 (E, H, H), b2 (E, H), w3 (E, H), b3 (E,)
    Values are float32 (the master-weight precision).
    """
    def u(shape, fan_in):
        lim = 1.0 / math.sqrt(fan_in)
        return rng.uniform(-lim, lim, size=shape).astype(np.float32)
    E, H = members, hidden
    return {
        "W1": u((E, H, d_in), d_in), "b1": u((E, H), d_in),
        "W2": u((E, H, H), H), "b2": u((E, H), H),
        "w3": u((E, H), H), "b3": u((E,), H),
    }


# --------------------------------------------------------------------------
# The paper's own 20-dimensional synthetic family (Sec. III-C, Fig. 1,
# Table I): four groups ("routines") of five parameters each on [-50, 50],
# Group 3 defined per case, the objective the sum of log |group output|.
# --------------------------------------------------------------------------

PAPER_BOUNDS = (-50.0, 50.0)
PAPER_GROUPS = [list(range(0, 5)), list(range(5, 10)), list(range(10, 15)), list(range(15, 20))]


def paper_groups(X, case, noise_std=0.0, rng=None):
    """Outputs of the four groups of the paper's synthetic function for the
    rows of X (..., 20), in the paper's notation:
      G1 = sum_{i=0}^{3} (x_i - x_{i+1})^2 + sum_{i=0}^{4} A_i
      G2 = sum_{k=5}^{8} (x_k - x_{k+1})^4 + sum_{k=5}^{9} A_k
      G3 = the Table I formula of the case (u = 10..14, v = 15..19; Cases 4
           and 5 pair v = u + 5)
      G4 = sum_{v=15}^{19} 1 / x_v
    with A_i = 10 cos(2 pi (x_i - 1)) + eps; eps ~ N(0, noise_std^2) on every
    A_i and once on each of G3 and G4.  Returns an array (..., 4)."""
    X = np.asarray(X, dtype=np.float64)
    shape = X.shape[:-1]

    def eps(k=1):
        if noise_std == 0.0:
            return 0.0
        return rng.normal(0.0, noise_std, size=shape + ((k,) if k > 1 else ()))

    def A(idx):
        a = 10.0 * np.cos(2.0 * math.pi * (X[..., idx] - 1.0))
        e = eps(len(idx))
        return np.sum(a + e, axis=-1)

    g1 = np.sum((X[..., 0:4] - X[..., 1:5]) ** 2, axis=-1) + A(list(range(0, 5)))
    g2 = np.sum((X[..., 5:9] - X[..., 6:10]) ** 4, axis=-1) + A(list(range(5, 10)))
    u = X[..., 10:15]
    v = X[..., 15:20]
    if case == 1:
        g3 = np.sum(u, axis=-1) + np.sum(np.cos(2.0 * math.pi * v), axis=-1)
    elif case == 2:
        g3 = np.sum(u * u, axis=-1) + np.sum(v, axis=-1)
    elif case == 3:
        g3 = np.sum(u * u, axis=-1) + np.sum(v * v, axis=-1)
    elif case == 4:
        g3 = np.sum((u * v ** 4) ** 2, axis=-1)
    elif case == 5:
        g3 = np.sum((u * v ** 8) ** 2, axis=-1)
    else:
        raise ValueError(f"case must be 1..5, got {case}")
    g3 = g3 + eps()
    g4 = np.sum(1.0 / v, axis=-1) + eps()
    return np.stack([g1, g2, g3, g4], axis=-1)


def paper_objective(X, case, noise_std=0.0, rng=None):
    """F = sum over the four groups of log |G_g| (the paper applies the log to
    the absolute value of each group's result)."""
    return np.sum(np.log(np.abs(paper_groups(X, case, noise_std, rng))), axis=-1)


def sensitivity_sweep(x0, V=100, step=1.1, bounds=PAPER_BOUNDS):
    """The configurations of the paper's one-at-a-time sensitivity sweep
    (Sec. IV-B): from the baseline x0 (d,), V variations per parameter, each
    multiplying the parameter by `step` relative to the preceding variation,
    clamped to the domain.  Returns (d, V, d): sweep[j, i] is x0 with
    parameter j at its (i+1)-th variation."""
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.shape[0]
    out = np.repeat(np.repeat(x0[None, None, :], V, axis=1), d, axis=0)
    for j in range(d):
        vals = x0[j] * step ** np.arange(1, V + 1)
        out[j, :, j] = np.clip(vals, bounds[0], bounds[1])
    return out


def make_paper_case(case, replicate=0, n=200, m=65536):
    """Observations and a candidate pool on the paper's family for one case:
    a baseline configuration for the sensitivity analysis, n uniform
    observations of F and m uniform candidates on [-50, 50]^20."""
    r_base, r_x, r_noise, r_c, _, _ = _streams(6, replicate * 8 + case)
    lo, hi = PAPER_BOUNDS
    x0 = f32r(r_base.uniform(lo, hi, size=20))
    X = f32r(r_x.uniform(lo, hi, size=(n, 20)))
    y = paper_objective(X, case, NOISE_STD, r_noise)
    Xc = f32r(r_c.uniform(lo, hi, size=(m, 20)))
    p = Problem(f"paper-case{case}", 20, X, y, Xc, np.full(20, 25.0), 1.0, NOISE_VAR, KERNEL_SE,
                None)
    p.extra["x0"] = x0
    p.extra["case"] = case
    return p


def make_config(name, replicate=0, **kw):
    if name == "c1":
        return make_c1(replicate, **kw)
    if name in ("c2", "c2-s"):
        return make_c2(replicate, scaled=name.endswith("-s"), **kw)
    if name in ("c5", "c5-s"):
        return make_c5(replicate, scaled=name.endswith("-s"), **kw)
    if name == "c4":
        return make_c4(replicate, **kw)
    raise KeyError(name)
