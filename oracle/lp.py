"""Deterministic arbitrage LP (Eq. (1) with separate charge/discharge).  TEST ONLY.

Variables per stage: c_t >= 0 (MWh bought from the grid), d_t >= 0 (MWh sold), and the
energy level e_t in [0, (S-1) delta] with
    e_t = e_{t-1} + eta_c c_t - d_t / eta_d,   e_0 = s0 delta,
    eta_c c_t <= W_c delta,   d_t / eta_d <= W_d delta          (per-stage SoC move limits),
objective  max sum_t lambda_t (d_t - c_t) - c_deg (d_t + c_t).
Without the complementarity binaries of Eq. (3) this is a relaxation of the storage
problem, so the discretised DP (a restriction, Sec. III-B) can never exceed it.  When
eta_c = eta_d = 1 and c_start = 0 the SoC constraints form an interval matrix (totally
unimodular), the LP has an optimum on the delta grid, and DP = LP.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog


def arbitrage_lp(st, lam, s0: int = 0):
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    T = lam.shape[0]
    cap = (st.S - 1) * st.delta
    n = 2 * T                                  # x = [c_1..c_T, d_1..d_T]
    cost = np.concatenate([lam + st.c_deg, -(lam - st.c_deg)])   # minimise -profit
    # cumulative energy e_t = e0 + sum_{u<=t} (eta_c c_u - d_u/eta_d) in [0, cap]
    L = np.tril(np.ones((T, T)))
    A = np.concatenate([st.eta_c * L, -(1.0 / st.eta_d) * L], axis=1)
    e0 = s0 * st.delta
    A_ub = np.concatenate([A, -A], axis=0)
    b_ub = np.concatenate([np.full(T, cap - e0), np.full(T, e0)])
    bounds = [(0.0, st.w_up * st.delta / st.eta_c)] * T + [(0.0, st.w_down * st.delta * st.eta_d)] * T
    res = linprog(cost, A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return -res.fun, res.x[:T], res.x[T:]
