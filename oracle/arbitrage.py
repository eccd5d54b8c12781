"""Continuous deterministic arbitrage of Eq. (1) and its reformulations.  TEST ONLY.

The perfect-foresight storage problem with net power p_t = p^d_t - p^c_t, energy level
s_t = s_{t-1} + eta p^c_t - p^d_t / eta (Eq. (2) written with the two directions of
Eq. (3b)), 0 <= s_t <= s_bar, 0 <= p^c_t, p^d_t <= p_bar and profit sum_t lam_t p_t
(hourly stages, MW x 1 h).  The variants compared with the DP in Sec. V:

* ``"exact"``    -- the MILP of Eq. (3a)-(3d): a binary z_t with p^c_t <= p_bar z_t and
                    p^d_t <= p_bar (1 - z_t), so charge and discharge never overlap;
* ``"relax"``    -- the same with z_t continuous in [0, 1] (the LP relaxation);
* ``"restrict"`` -- no z, and p^d_t = 0 wherever lam_t <= 0 (the LP restriction);
* ``"lp"``       -- no z and no restriction (the plain LP, used as the upper bound in the
                    deterministic accuracy study).

Sparse constraint matrices, solved by HiGHS through ``scipy.optimize.milp``.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse
from scipy.optimize import Bounds, LinearConstraint, milp

MODES = ("exact", "relax", "restrict", "lp")


def arbitrage(lam, *, s_bar: float, p_bar: float, eta: float, s0: float, mode: str = "exact"):
    """Return dict(profit, pc, pd, s, overlap) for the chosen formulation.

    overlap = fraction of stages with p^c_t p^d_t > 1e-9 (simultaneous charge/discharge).
    """
    if mode not in MODES:
        raise ValueError(mode)
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    T = lam.shape[0]
    use_z = mode in ("exact", "relax")
    nz = T if use_z else 0
    n = 3 * T + nz                              # x = [pc (T), pd (T), s (T), z (nz)]
    ipc, ipd, isv, iz = 0, T, 2 * T, 3 * T
    c = np.zeros(n)
    c[ipc:ipc + T] = lam                        # minimise -profit = sum lam (pc - pd)
    c[ipd:ipd + T] = -lam
    rows, cols, vals = [], [], []
    t = np.arange(T)
    # energy balance: s_t - s_{t-1} - eta pc_t + pd_t / eta = 0  (s_0 on the right-hand side)
    rows += [t, t, t]
    cols += [isv + t, ipc + t, ipd + t]
    vals += [np.ones(T), np.full(T, -eta), np.full(T, 1.0 / eta)]
    rows.append(t[1:])
    cols.append(isv + t[1:] - 1)
    vals.append(-np.ones(T - 1))
    lb = np.zeros(T)
    ub = np.zeros(T)
    lb[0] = ub[0] = s0
    nrow = T
    if use_z:
        # pc_t - p_bar z_t <= 0 ;  pd_t + p_bar z_t <= p_bar
        r1 = nrow + t
        r2 = nrow + T + t
        rows += [r1, r1, r2, r2]
        cols += [ipc + t, iz + t, ipd + t, iz + t]
        vals += [np.ones(T), np.full(T, -p_bar), np.ones(T), np.full(T, p_bar)]
        lb = np.concatenate([lb, np.full(2 * T, -np.inf)])
        ub = np.concatenate([ub, np.zeros(T), np.full(T, p_bar)])
        nrow += 2 * T
    A = sparse.csr_array((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nrow, n))
    lo = np.zeros(n)
    hi = np.concatenate([np.full(2 * T, p_bar), np.full(T, s_bar), np.ones(nz)])
    if mode == "restrict":
        hi[ipd:ipd + T] = np.where(lam <= 0.0, 0.0, p_bar)
    integrality = np.zeros(n)
    if mode == "exact":
        integrality[iz:iz + T] = 1
    res = milp(c, constraints=LinearConstraint(A, lb, ub), integrality=integrality,
               bounds=Bounds(lo, hi), options={"mip_rel_gap": 1e-9})
    if res.x is None:
        raise RuntimeError(res.message)
    x = res.x
    pc, pd, s = x[ipc:ipc + T], x[ipd:ipd + T], x[isv:isv + T]
    return {"profit": float(lam @ (pd - pc)), "pc": pc, "pd": pd, "s": s,
            "overlap": float(np.mean(pc * pd > 1e-9))}
