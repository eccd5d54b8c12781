"""Exhaustive plan enumeration on tiny scenario trees (FP64).  TEST INFRASTRUCTURE ONLY.

A non-anticipative plan fixes one next-SoC index j for every node of the price
scenario tree (a node is the history of observed price states k_1 .. k_t).  This
module lists *every* feasible plan explicitly and evaluates its expected profit by
summing over every price path with its probability, then takes the maximum.  No
backward induction is used, so agreement with the DP value of Eq. (5)-(6) checks
the recursion itself (Bellman's principle on the tree), not a re-typed copy of it.
"""
from __future__ import annotations

import itertools

import numpy as np


def _g(st, d):
    if d > 0:
        return -d * st.delta / st.eta_c
    if d < 0:
        return -d * st.delta * st.eta_d
    return 0.0


def _r(st, lam, d):
    g = _g(st, d)
    return lam * g - st.c_deg * abs(g) - (st.c_start if d != 0 else 0.0)


def _feasible(st, s):
    return range(max(0, s - st.w_down), min(st.S - 1, s + st.w_up) + 1)


def _plans(st, T, K, t, s, hist):
    """All plans of the subtree at node ``hist`` (stage t, SoC s): list of dicts."""
    out = []
    for j in _feasible(st, s):
        if t == T:
            out.append({hist: j})
            continue
        child_lists = [_plans(st, T, K, t + 1, j, hist + (kk,)) for kk in range(K)]
        for combo in itertools.product(*child_lists):
            plan = {hist: j}
            for c in combo:
                plan.update(c)
            out.append(plan)
    return out


def _evaluate(st, lam, P, v_term, plan, s0, k0):
    T, K = lam.shape
    total = 0.0
    for tail in itertools.product(range(K), repeat=T):      # k_2 .. k_{T+1}
        path = (k0,) + tail
        prob = 1.0
        for t in range(1, T + 1):                           # P_t links k_t -> k_{t+1}
            prob *= float(P[t - 1, path[t - 1], path[t]])
        if prob == 0.0:
            continue
        s, val = s0, 0.0
        for t in range(1, T + 1):
            j = plan[path[:t]]
            val += _r(st, float(lam[t - 1, path[t - 1]]), j - s)
            s = j
        if v_term is not None:
            val += float(v_term[path[T], s])
        total += prob * val
    return total


def best_plan_value(st, lam, P, s0: int, k0: int, v_term=None):
    """max over all non-anticipative plans of the expected profit from (s0, k0)."""
    lam = np.asarray(lam, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    T, K = lam.shape
    plans = _plans(st, T, K, 1, s0, (k0,))
    best = -np.inf
    for plan in plans:
        v = _evaluate(st, lam, P, v_term, plan, s0, k0)
        if v > best:
            best = v
    return best, len(plans)


def best_markov_policy_value(st, lam, P, s0: int, k0: int):
    """max over every deterministic Markov policy (t, s, k) -> j, evaluated by path sums."""
    lam = np.asarray(lam, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    T, K = lam.shape
    keys = [(t, s, k) for t in range(1, T + 1) for s in range(st.S) for k in range(K)]
    choices = [list(_feasible(st, s)) for (_, s, _) in keys]
    best = -np.inf
    for combo in itertools.product(*choices):
        pol = dict(zip(keys, combo))
        total = 0.0
        for tail in itertools.product(range(K), repeat=T - 1):
            path = (k0,) + tail
            prob = 1.0
            for t in range(1, T):
                prob *= float(P[t - 1, path[t - 1], path[t]])
            s, val = s0, 0.0
            for t in range(1, T + 1):
                j = pol[(t, s, path[t - 1])]
                val += _r(st, float(lam[t - 1, path[t - 1]]), j - s)
                s = j
            total += prob * val
        best = max(best, total)
    return best
