"""Algorithm 1 (tensor-based backward induction) with NumPy, FP64.  TEST ONLY.

The stagewise-independent model of Sec. II-B: prices lambda_t take R sampled levels
with probabilities pi_t, the value function V_t(s) depends on SoC only.  The steps
follow Algorithm 1 in order: next-state levels sigma (outer sum of the SoC grid and
F of the power grid), projection onto [0, s_bar] and index proxies, floor/ceil
indices, interpolation factors, then per stage the interpolated gather, the -inf
mask of infeasible pairs, the S x P x R payoff tensor, the max over actions and the
expectation.

Readings of garbled or silent points (each also listed in the design notes):
* the projection of sigma is onto [0, s_bar] (the text says so; the printed formula
  swaps min and max);
* indices are 0-based here, so the proxy is z = clip(sigma, 0, s_bar) / delta;
* the interpolation factor is 0 where floor and ceil coincide;
* a pair is infeasible when sigma < 0 or sigma > s_bar (the printed test compares
  with S, a count, not an energy); a relative slack of 1e-9 s_bar absorbs rounding;
* the loop runs t = T..1 and returns V_{T-1} .. V_0;
* the last entry of F(p_hat) is -p_bar / eta (its sign is lost in print).
"""
from __future__ import annotations

import math

import numpy as np


def soc_grid(duration_h: float, delta: float, p_bar: float = 1.0):
    """s_hat = [0, delta, ..., s_bar] with S = s_bar / delta + 1 (Sec. III-A)."""
    n = int(round(duration_h * p_bar / delta))
    return np.arange(n + 1, dtype=np.float64) * delta


def power_grid(p_bar: float, delta: float, eta: float):
    """Recombining action vector p_hat of Sec. III-A, ascending.

    n_c = ceil(p_bar eta / delta) charging actions -k delta / eta (the last one is the
    endpoint -p_bar), n_d = ceil(p_bar / (delta eta)) discharging actions k delta eta
    (the last one is +p_bar), plus 0; P = n_c + n_d + 1.
    """
    n_c = math.ceil(p_bar * eta / delta - 1e-12)
    n_d = math.ceil(p_bar / (delta * eta) - 1e-12)
    charge = [-(k * delta / eta) for k in range(1, n_c)] + [-p_bar]
    discharge = [k * delta * eta for k in range(1, n_d)] + [p_bar]
    p = np.array(sorted(charge) + [0.0] + discharge, dtype=np.float64)
    return p, n_c, n_d


def F(p: np.ndarray, eta: float) -> np.ndarray:
    """State transition of Eq. (2): -p / eta when discharging (p >= 0), -eta p when charging."""
    p = np.asarray(p, dtype=np.float64)
    return np.where(p >= 0, -p / eta, -eta * p)


def precompute(s_hat, p_hat, eta: float):
    """Algorithm 1's stage-invariant steps: next-state levels, proxies, indices, factors."""
    s_hat = np.asarray(s_hat, dtype=np.float64)
    p_hat = np.asarray(p_hat, dtype=np.float64)
    delta = s_hat[1] - s_hat[0]
    s_bar = s_hat[-1]
    sigma = s_hat[:, None] + F(p_hat, eta)[None, :]                       # S x P
    z = np.clip(sigma, 0.0, s_bar) / delta
    z_lo = np.floor(z + 1e-9).astype(np.int64)
    z_hi = np.ceil(z - 1e-9).astype(np.int64)
    z_lo = np.minimum(z_lo, z_hi)
    span = (z_hi - z_lo).astype(np.float64)
    b = np.where(span > 0, (z - z_lo) / np.where(span > 0, span, 1.0), 0.0)
    tol = 1e-9 * s_bar
    infeasible = (sigma < -tol) | (sigma > s_bar + tol)
    return z_lo, z_hi, b, infeasible


def stage(pre, p_hat, lam_t, pi_t, V_t, rows=None):
    """One iteration of the loop: returns (V_{t-1} [S or rows], Q_all [S|rows, P, R]).

    ``rows`` restricts the computation to some SoC indices (memory only; every row is
    computed independently of the others)."""
    z_lo, z_hi, b, infeasible = pre
    if rows is not None:
        z_lo, z_hi, b, infeasible = z_lo[rows], z_hi[rows], b[rows], infeasible[rows]
    V_t = np.asarray(V_t, dtype=np.float64)
    Vn = (1.0 - b) * V_t[z_lo] + b * V_t[z_hi]                             # S x P
    Vn = np.where(infeasible, -np.inf, Vn)
    Q_all = np.outer(np.asarray(p_hat, np.float64),
                     np.asarray(lam_t, np.float64))[None, :, :] + Vn[:, :, None]   # S x P x R
    Q = Q_all.max(axis=1)                                                  # S x R
    return Q @ np.asarray(pi_t, np.float64), Q_all


def policy_index(Q_all):
    """Maximising action per (s, r) with ties resolved to the largest index: the largest
    power sold, i.e. the smallest next state (the convention of the grid-DP policy, where
    a tie goes to the smallest next SoC)."""
    P = Q_all.shape[1]
    return P - 1 - np.argmax(Q_all[:, ::-1, :], axis=1)                   # S x R


def algorithm1(s_hat, p_hat, lam, pi, eta: float):
    """Return the expected value vectors V_hat [T+1, S] with V_hat[T] = 0.

    lam, pi: [T, R] sampled levels and probabilities for stages t = 1..T.
    """
    lam = np.asarray(lam, dtype=np.float64)
    pi = np.asarray(pi, dtype=np.float64)
    T, R = lam.shape
    S = np.asarray(s_hat).shape[0]
    pre = precompute(s_hat, p_hat, eta)
    V = np.zeros((T + 1, S))
    for t in range(T, 0, -1):
        V[t - 1], _ = stage(pre, p_hat, lam[t - 1], pi[t - 1], V[t])
    return V
