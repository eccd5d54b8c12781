"""Bids of the paper mode and their merit-order clearing (Sec. II-C, Sec. V-A); host, FP64.

Works on the expected values V_t (t = 0..T, [T+1, S]) that ``solve_independent`` returns
with ``store_all=True``.  The bid of stage t at an incoming energy level s (any real value
in [0, s_bar], not only a grid point) offers every feasible power p of Eq. (4) with the
continuation value

    U_t(p; s) = V_t(s + F(p)),     F(p) = -p / eta (p >= 0),  -eta p (p < 0)     (Eq. (7))

and V_t linearly interpolated between grid levels.  The bid is b~ = -dU~/dp of the concave
envelope U~ (Eq. (9)-(10)), built with the monotone-chain hull of ``bids.upper_hull``.  A
price-taker storage facing the realised price lam clears the quantity where lam meets the
bid: the envelope vertex maximising lam p + U~(p) (the largest quantity on a tie).  The
simulation walks t = 1..T, clears each stage's bid at its realised price, earns lam_t p_t
and moves to s + F(p_t).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import numpy as np

from . import _lib
from .bids import upper_hull


@dataclasses.dataclass
class PaperGrid:
    S: int
    delta: float
    eta: float
    p_bar: float
    p: np.ndarray            # ascending power grid p_hat (MW; > 0 sells)

    @property
    def s_bar(self) -> float:
        return (self.S - 1) * self.delta


def paper_grid(S: int, delta: float, eta: float, p_bar: float) -> PaperGrid:
    """The recombining grid of Sec. III-A for the FP32 parameters the GPU solve uses.

    The action counts come from the library (``dp_iid_action_grid``), so the host grid is
    the one the solve maximised over: n_c - 1 interior charge actions -k delta / eta, the
    charge endpoint -p_bar, 0, n_d - 1 interior discharge actions k delta eta and p_bar.
    """
    f = lambda x: float(np.float32(x))
    pb = _lib.IidProblem(T=1, R=1, S=int(S), reserved=0, delta=f(delta), eta=f(eta),
                         p_bar=f(p_bar), flags=0)
    P, n_c, n_d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.lib().dp_iid_action_grid(ctypes.byref(pb), ctypes.byref(P), ctypes.byref(n_c),
                                             ctypes.byref(n_d)))
    d, e, pbar = f(delta), f(eta), f(p_bar)
    charge = [-pbar] + [-(k * d / e) for k in range(n_c.value - 1, 0, -1)]
    discharge = [k * d * e for k in range(1, n_d.value)] + [pbar]
    p = np.array(charge + [0.0] + discharge, dtype=np.float64)
    assert p.shape[0] == P.value
    return PaperGrid(int(S), d, e, pbar, p)


def transition(p, eta: float):
    """F(p) of Eq. (2): the change of stored energy for net power p."""
    p = np.asarray(p, dtype=np.float64)
    return np.where(p >= 0.0, -p / eta, -eta * p)


def value_at(V_t: np.ndarray, x, delta: float):
    """V_t at energy levels x in [0, s_bar] by linear interpolation between grid levels."""
    V_t = np.asarray(V_t, dtype=np.float64)
    grid = np.arange(V_t.shape[0], dtype=np.float64) * delta
    return np.interp(np.asarray(x, dtype=np.float64), grid, V_t)


@dataclasses.dataclass
class PaperBid:
    p: np.ndarray            # feasible quantities, ascending
    U: np.ndarray            # U_t(p; s)
    nxt: np.ndarray          # next energy level of each quantity
    hull: np.ndarray         # envelope vertices (indices into p), ascending

    def segments(self):
        """(p_lo, p_hi, price) per envelope segment; prices non-decreasing in p."""
        h = self.hull
        return [(float(self.p[a]), float(self.p[b]),
                 float(-(self.U[b] - self.U[a]) / (self.p[b] - self.p[a])))
                for a, b in zip(h[:-1], h[1:])]

    def clear(self, price: float):
        """(quantity, next level, stage profit price * quantity) cleared at a price."""
        h = self.hull
        obj = price * self.p[h] + self.U[h]
        i = h[np.flatnonzero(obj == np.max(obj))[-1]]
        return float(self.p[i]), float(self.nxt[i]), float(price * self.p[i])


def bid(V_t: np.ndarray, s: float, grid: PaperGrid) -> PaperBid:
    """The convexified bid of a stage whose expected next-stage values are V_t.

    The offered quantities are the continuous interval of Eq. (4),
    [max(-p_bar, -(s_bar - s) / eta), min(p_bar, s eta)].  On it U(p) = V_t(s + F(p)) is
    piecewise linear, with breakpoints where s + F(p) meets a grid level, at p = 0 (the kink
    of F) and at the interval ends, so those points carry the whole curve and its envelope.
    From a grid level they are exactly the grid actions the DP maximised over.
    """
    sb, d, eta, pb = grid.s_bar, grid.delta, grid.eta, grid.p_bar
    tol = 1e-9 * max(1.0, sb)
    lo = max(0.0, s - pb / eta)                  # lowest reachable level (full discharge)
    hi = min(sb, s + eta * pb)                   # highest reachable level (full charge)
    j = np.arange(math.ceil(lo / d - 1e-9), math.floor(hi / d + 1e-9) + 1)
    x = np.concatenate([j * d, [lo, hi, s]])
    x = np.clip(x, 0.0, sb)
    x = np.sort(x)[::-1]                         # descending level = ascending quantity
    keep = np.concatenate([[True], np.diff(x) < -tol])
    x = x[keep]
    p = np.where(x <= s, (s - x) * eta, -(x - s) / eta)
    U = value_at(V_t, x, d)
    return PaperBid(p, U, x, upper_hull(p, U))


def simulate_bidding(V_all: np.ndarray, lam, s0: float, grid: PaperGrid):
    """Clear the bids of stages 1..T at the realised prices lam[0..T-1] from level s0.

    V_all[t] is the expected value after stage t (V_all[T] = terminal).  Returns
    dict(profit, p [T], s [T+1]).
    """
    V_all = np.asarray(V_all, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    T = lam.shape[0]
    if V_all.shape[0] != T + 1:
        raise ValueError("V_all must hold T + 1 value vectors")
    s = np.empty(T + 1)
    p = np.empty(T)
    s[0] = s0
    profit = 0.0
    for t in range(1, T + 1):
        b = bid(V_all[t], s[t - 1], grid)
        p[t - 1], s[t], earned = b.clear(float(lam[t - 1]))
        profit += earned
    return {"profit": profit, "p": p, "s": s}
