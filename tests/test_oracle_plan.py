"""Pins of the interdependence-analysis oracle (oracle/plan.py) against what
the paper and the mathematics fix: zero cross-routine influence for an
additively separable objective, growth with the coupling strength, the
qualitative ordering of the paper's Table II on its synthetic family, the
paper's search sets for its five cases (Sec. IV-D: Group 3 and Group 4
merged in Cases 3, 4 and 5, all four groups independent in Cases 1 and 2),
and the dimension cap against a brute-force choice."""
import itertools

import numpy as np
import pytest

from oracle import plan as PL
from paper_2403_08131_amd import inputs as I

OWNER20 = [j // 5 for j in range(20)]


def _baseline_groups(X, spec):
    """Per-group outputs of the baseline family: each group's own terms plus
    the chain coupling to the next group's first variable."""
    X = np.asarray(X, dtype=np.float64)
    G = len(spec.groups)
    outs = []
    for g, idx in enumerate(spec.groups):
        sub = I.SyntheticSpec(groups=[idx], pair_coef=spec.pair_coef, lam=0.0)
        o = I.synthetic_f(X, sub)
        if g + 1 < G:
            o = o + spec.lam * np.cos(np.pi * (X[..., idx[0]] - X[..., spec.groups[g + 1][0]]))
        outs.append(o)
    return np.stack(outs, axis=-1)


def _sweep_S(groups_fn, x0, V=40, step=1.1, bounds=(0.05, 1.0)):
    sw = I.sensitivity_sweep(x0, V=V, step=step, bounds=bounds)
    return PL.sensitivity(groups_fn(x0), groups_fn(sw))


def test_sensitivity_definition_small_case():
    base = np.array([2.0, -4.0])
    out = np.array([[[3.0, -4.0], [1.0, -2.0]]])  # P = 1, V = 2, R = 2
    S = PL.sensitivity(base, out)
    assert S[0, 0] == pytest.approx((0.5 + 0.5) / 2)
    assert S[1, 0] == pytest.approx((0.0 + 0.5) / 2)


def test_separable_objective_has_zero_external_influence():
    spec = I.spec_grouped(20, 0.0)
    x0 = np.random.default_rng(3).uniform(0.1, 0.5, 20)
    S = _sweep_S(lambda X: _baseline_groups(X, spec), x0)
    for r in range(4):
        for j in range(20):
            if OWNER20[j] != r:
                assert S[r, j] == 0.0, (r, j)
    rs, ps, n = PL.plan(S, OWNER20)
    assert n == 4 and list(rs) == [0, 1, 2, 3]


def test_external_influence_grows_with_coupling():
    x0 = np.random.default_rng(4).uniform(0.1, 0.5, 20)
    prev = 0.0
    for lam in (0.05, 0.2, 0.5, 1.0):
        spec = I.spec_grouped(20, lam)
        S = _sweep_S(lambda X: _baseline_groups(X, spec), x0)
        ext = S[0, 5]  # group 0 through the next group's first variable
        assert ext > prev
        prev = ext
        assert S[0, 6] == 0.0  # other variables of the next group stay out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_table2_ordering_and_paper_search_sets(seed):
    """Group 3's sensitivity to Group 4 variables, relative to its own: very
    low (Case 1) and low (Case 2) below the cut-off, comparable (Case 3) and
    dominant (Cases 4, 5) above it; the resulting search sets are the
    paper's."""
    r = np.random.default_rng(1000 + seed)
    x0 = I.f32r(r.uniform(-50, 50, 20))
    sw = I.sensitivity_sweep(x0)
    ratios = []
    # evaluation noise small against every group's scale (Group 4 is a sum
    # of reciprocals and can be ~1e-2): the paper reports the noise's share
    # of the variability below 1 %
    noise = 1e-5
    for case in range(1, 6):
        base = I.paper_groups(x0, case, noise, r)
        out = I.paper_groups(sw, case, noise, r)
        S = PL.sensitivity(base, out)
        own = S[2, 10:15].max()
        ext = S[2, 15:20].max()
        ratios.append(ext / own)
        rs, ps, n = PL.plan(S, OWNER20, cutoff=0.25)
        if case in (1, 2):
            assert n == 4 and list(rs) == [0, 1, 2, 3], case
        else:
            assert n == 3 and list(rs) == [0, 1, 2, 2], case
        assert list(ps) == [rs[o] for o in OWNER20]  # 10 parameters: no cap
        # no external influence on Groups 1, 2 and 4 beyond the noise
        for g in (0, 1, 3):
            ext_g = max(S[g, j] for j in range(20) if OWNER20[j] != g)
            assert ext_g <= 0.01 * S[g, [j for j in range(20) if OWNER20[j] == g]].max(), (case, g)
    assert ratios[0] < 0.25 and ratios[1] < 0.25
    assert 0.25 <= ratios[2] <= 4.0
    assert ratios[3] > 1.0 and ratios[4] > ratios[3]


def test_cap_keeps_the_most_influential_parameters():
    """A merged search of 15 parameters is cut to 10 by influence; compared
    with a brute force over all 10-subsets of the largest total influence."""
    rng = np.random.default_rng(7)
    owner = [0] * 5 + [1] * 5 + [2] * 5
    S = rng.uniform(0.05, 1.0, (3, 15))
    S[0, 5] = S[1, 10] = 2.0  # routine 1 depends on routine 0's... chain 0-1-2
    rs, ps, n = PL.plan(S, owner, cutoff=0.25, max_dims=10)
    assert n == 1
    Iinf = PL.influence(S, owner)
    score = Iinf.max(axis=0)
    best = max(itertools.combinations(range(15), 10), key=lambda c: (sum(score[list(c)]), [-j for j in c]))
    assert sorted(np.flatnonzero(ps >= 0)) == sorted(best)
