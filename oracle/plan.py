"""Plain reference of the interdependence analysis that decides the set of
tuning searches (the paper's Sec. IV-B to IV-D).  TEST INFRASTRUCTURE ONLY:
the tests import it; the product path never does, and it shares no code with
the library's planner.

Steps, in the paper's order:

1. Sensitivity (Sec. IV-B): from a baseline configuration, V variations of
   one parameter at a time; the sensitivity of routine r to parameter j is
   the mean relative change of the routine's output,
       S[r, j] = (1/V) sum_i |(out_r(base) - out_r(variation i of j)) / out_r(base)|.
2. Influence score (Sec. IV-C): the sensitivity relative to the routine's
   most sensitive own parameter (reading: the paper quotes absolute
   variabilities, which depend on the baseline and on how far the sweep can
   move a parameter; the relative score makes one cut-off apply to routines
   of any output scale),
       I[r, j] = S[r, j] / max_{j' owned by r} S[r, j'].
3. Graph and cut-off (Sec. IV-C): parameter j is an edge from its own
   routine to every routine r with I[r, j] >= cut-off; weaker edges are
   pruned.
4. Searches (Sec. IV-D): routines joined by a path of kept edges are tuned
   in one merged search; here the connected components are found by a
   breadth-first search over routines.
5. Dimension cap (Sec. IV-D): a search with more than `max_dims` parameters
   keeps the most influential ones (largest influence on any routine of the
   search; ties to the lower index) and fixes the rest at their defaults.

Parity status: pinned in tests/test_oracle_plan.py (zero influence for an
additively separable function, the qualitative ordering of the paper's
Table II, the paper's search sets for its five synthetic cases, a brute-force
cap).
"""
from __future__ import annotations

import numpy as np


def sensitivity(base, out):
    """base: (R,) routine outputs at the baseline; out: (P, V, R) outputs at
    the V variations of each of the P parameters.  Returns S (R, P)."""
    base = np.asarray(base, dtype=np.float64)
    out = np.asarray(out, dtype=np.float64)
    P, V, R = out.shape
    S = np.zeros((R, P))
    for r in range(R):
        for j in range(P):
            acc = 0.0
            for i in range(V):
                acc += abs((base[r] - out[j, i, r]) / base[r])
            S[r, j] = acc / V
    return S


def influence(S, owner):
    """I[r, j] = S[r, j] / (largest S[r, j'] over the parameters j' of r)."""
    R, P = S.shape
    I = np.zeros_like(S)
    for r in range(R):
        own = [S[r, j] for j in range(P) if owner[j] == r]
        top = max(own) if own else 0.0
        for j in range(P):
            I[r, j] = S[r, j] / top if top > 0.0 else 0.0
    return I


def plan(S, owner, cutoff=0.25, max_dims=10):
    """Returns (routine_search (R,), param_search (P,), n_searches): the
    search of every routine (numbered in order of each search's lowest
    routine), and of every parameter (-1 when dropped by the cap)."""
    S = np.asarray(S, dtype=np.float64)
    R, P = S.shape
    I = influence(S, owner)
    # adjacency between routines through kept external edges
    adj = [set() for _ in range(R)]
    for j in range(P):
        o = owner[j]
        for r in range(R):
            if r != o and I[r, j] >= cutoff:
                adj[o].add(r)
                adj[r].add(o)
    routine_search = [-1] * R
    n = 0
    for r0 in range(R):
        if routine_search[r0] >= 0:
            continue
        queue = [r0]
        routine_search[r0] = n
        while queue:
            r = queue.pop(0)
            for q in sorted(adj[r]):
                if routine_search[q] < 0:
                    routine_search[q] = n
                    queue.append(q)
        n += 1
    param_search = [routine_search[owner[j]] for j in range(P)]
    for s in range(n):
        members = [j for j in range(P) if param_search[j] == s]
        if len(members) <= max_dims:
            continue
        routines = [r for r in range(R) if routine_search[r] == s]
        score = {j: max(I[r, j] for r in routines) for j in members}
        keep = sorted(members, key=lambda j: (-score[j], j))[:max_dims]
        for j in members:
            if j not in keep:
                param_search[j] = -1
    return np.array(routine_search), np.array(param_search), n
