"""Comparison rules between the HIP path and the FP64 oracle (shared by the GPU tests).

Values: per stage, max_{k,s} |V_gpu - V_or| <= RTOL * max_{k,s} |V_or| (normwise; an
elementwise relative test is meaningless where V crosses 0).  RTOL = 1e-5.

Policies: identical, except at near-ties: a mismatch at (t, k, s) is accepted iff the
oracle's own Q value of the GPU's choice is within RTOL * max|V_or,t| of the oracle's
maximum (FP32 and FP64 may order two candidates that close differently).  Every
accepted mismatch is counted and reported.
"""
from __future__ import annotations

import numpy as np

import oracle

RTOL = 1e-5


def value_error(v_gpu: np.ndarray, v_or: np.ndarray) -> float:
    scale = max(float(np.max(np.abs(v_or))), 1e-30)
    return float(np.max(np.abs(v_gpu.astype(np.float64) - v_or))) / scale


def check_stage(st, lam_t, P_t, v_next_or, v_gpu, pol_gpu, *, label=""):
    """Compare one stage's GPU values and policies against the oracle stage computed from
    v_next_or (the FP64 V_{t+1}).  Returns the number of accepted near-tie mismatches."""
    v_or, pol_or, _ = oracle.stage(st, lam_t, P_t, v_next_or, want_w=True)
    err = value_error(v_gpu, v_or)
    assert err <= RTOL, f"{label}: normwise value error {err:.3e} > {RTOL}"
    if np.array_equal(pol_gpu, pol_or):
        return 0
    return _mismatch(st, lam_t, P_t, v_next_or, v_or, pol_gpu, pol_or, label)


def check_solve(st, lam, P, V_gpu_all, pol_gpu, or_out, label=""):
    """Full-solve comparison, stage by stage; returns total accepted mismatches."""
    T = lam.shape[0]
    V_or = or_out["V"]
    pol_or = or_out["policy"]
    total = 0
    for t in range(T, 0, -1):
        err = value_error(V_gpu_all[t - 1], V_or[t - 1])
        assert err <= RTOL, f"{label} stage {t}: normwise value error {err:.3e}"
        if not np.array_equal(pol_gpu[t - 1], pol_or[t - 1]):
            total += _mismatch(st, lam[t - 1], P[t - 1], V_or[t], V_or[t - 1], pol_gpu[t - 1],
                               pol_or[t - 1], f"{label} stage {t}")
    return total


STATS = {"mismatch": 0, "max_regret": 0.0}


def _mismatch(st, lam_t, P_t, v_next_or, v_or, pol_gpu, pol_or, label, W=None):
    if W is None:
        _, _, W = oracle.stage(st, lam_t, P_t, v_next_or, want_w=True)
    scale = max(float(np.max(np.abs(v_or))), 1e-30)
    tol = RTOL * scale
    k, s = np.nonzero(pol_gpu != pol_or)
    STATS["mismatch"] += int(k.size)
    if k.size == 0:
        return 0
    j = pol_gpu[k, s].astype(np.int64)
    q = oracle.q_at(st, lam_t, W, k, s, j)
    bad = ~np.isfinite(q)
    assert not bad.any(), (f"{label}: GPU chose an infeasible move at k={k[bad][0]}, "
                           f"s={s[bad][0]} (j={j[bad][0]})")
    regret = v_or[k, s] - q
    i = int(np.argmax(regret))
    assert regret[i] <= tol, (
        f"{label}: policy mismatch at k={k[i]} s={s[i]}: gpu j={j[i]} (Q={q[i]:.9g}) vs "
        f"oracle j={int(pol_or[k[i], s[i]])} (V={v_or[k[i], s[i]]:.9g})")
    STATS["max_regret"] = max(STATS["max_regret"], float(regret[i]) / scale)
    return int(k.size)
