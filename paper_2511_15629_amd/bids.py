"""Price-quantity bid curves from the solved DP (Sec. II-C, Eq. (7)-(10)); host, FP64.

For a stage t, incoming state of charge s and observed price state k, every feasible move
d = j - s sells p(d) = g(d) MWh to the grid and leaves the continuation value

    U(p) = h(d) + W_t[k][s + d],      h(d) = -c_deg |g(d)| - c_start [d != 0],

where W_t = P_t V_{t+1} is the expected next-stage value and h the price-independent part
of the payoff (zero in the paper's linear case, so U(p) = V_t(s + F(p)) as in Eq. (7)).
At a market price lam the storage earns lam p + U(p).  When U is not concave (start costs,
negative prices) the bid uses the concave envelope U~ whose hypograph is the convex hull
of the hypograph of U (Eq. (9)); the monotone bid is b~(p) = -dU~/dp (Eq. (10)).  The hull
is built with Andrew's monotone chain (a Graham-scan variant), O(n) on points already
ordered by p.

For every price lam, max_p lam p + U~(p) = max_p lam p + U(p): the envelope changes which
quantities are offered, never the optimal profit.  The quantity cleared at lam is the hull
vertex maximising lam p + U~(p) (the largest such quantity on a tie, the supply-curve
convention).

Markov prices.  The bid for stage t is decided at t - 1, before the price state k of stage
t is known (Sec. II-C), but here the continuation W_t[k] depends on k, which the price
itself reveals: the curve of state k applies when the price is lam_t[k].  Each state's
curve gives the quantity q_k it clears at its own level lam_t[k]; the bid submitted for
(t, s) is the price-sorted monotone envelope of the points (lam_t[k], q_k): at the level
of state k it offers max{q_k' : lam_t[k'] <= lam_t[k]}, the least non-decreasing supply
schedule that offers at least q_k at every level (market rules require a non-decreasing
curve).  Where the q_k are already non-decreasing in price (always so with independent
prices, where every state has the same concave U~) the envelope offers exactly q_k and
clears the DP's value; elsewhere it gives up the difference, which `MarkovBid` reports.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


def move_energy(storage, d: np.ndarray) -> np.ndarray:
    """MWh sold to the grid by a move of d grid steps (Eq. (2) on the recombining grid)."""
    d = np.asarray(d, dtype=np.float64)
    up = -d * storage.delta / storage.eta_c
    down = -d * storage.delta * storage.eta_d
    return np.where(d > 0, up, np.where(d < 0, down, 0.0))


@dataclasses.dataclass
class BidCurve:
    p: np.ndarray        # quantities (MWh sold), ascending
    U: np.ndarray        # continuation value of each quantity (incl. price-free payoff)
    j: np.ndarray        # next-state index reached by each quantity
    hull: np.ndarray     # indices of the upper-hull vertices, ascending in p

    def segments(self):
        """Monotone bid: list of (p_lo, p_hi, price) with price = -slope of U~ on the
        segment; prices are non-decreasing in p."""
        out = []
        h = self.hull
        for a, b in zip(h[:-1], h[1:]):
            slope = (self.U[b] - self.U[a]) / (self.p[b] - self.p[a])
            out.append((float(self.p[a]), float(self.p[b]), float(-slope)))
        return out

    def envelope(self, x) -> np.ndarray:
        """U~ at quantities x (piecewise-linear through the hull vertices)."""
        hp, hu = self.p[self.hull], self.U[self.hull]
        return np.interp(np.asarray(x, dtype=np.float64), hp, hu)

    def clear(self, price: float):
        """Quantity, next state and profit cleared at a market price."""
        h = self.hull
        obj = price * self.p[h] + self.U[h]
        best = np.max(obj)
        idx = h[np.flatnonzero(obj == best)[-1]]
        return float(self.p[idx]), int(self.j[idx]), float(best)


def upper_hull(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Indices of the upper convex hull of points sorted by strictly increasing x."""
    stack: List[int] = []
    for i in range(x.shape[0]):
        while len(stack) >= 2:
            a, b = stack[-2], stack[-1]
            cross = (x[b] - x[a]) * (y[i] - y[a]) - (y[b] - y[a]) * (x[i] - x[a])
            if cross >= 0:          # b lies on or below the chord a -> i
                stack.pop()
            else:
                break
        stack.append(i)
    return np.asarray(stack, dtype=np.int64)


def bid_curve(w_row: np.ndarray, s: int, storage) -> BidCurve:
    """Bid curve at SoC index s from one row W_t[k][.] of expected next-stage values."""
    w_row = np.asarray(w_row, dtype=np.float64)
    S = int(storage.S)
    lo, hi = max(0, s - int(storage.w_down)), min(S - 1, s + int(storage.w_up))
    j = np.arange(hi, lo - 1, -1)            # descending j = ascending quantity sold
    d = j - s
    p = move_energy(storage, d)
    g = np.abs(p)
    h = -float(storage.c_deg) * g - float(storage.c_start) * (d != 0)
    U = h + w_row[j]
    return BidCurve(p=p, U=U, j=j, hull=upper_hull(p, U))


def expectation_row(V_next: np.ndarray, P_t: np.ndarray, k: int) -> np.ndarray:
    """W_t[k][.] = sum_k' P_t[k][k'] V_{t+1}[k'][.] in FP64 on the host."""
    return np.asarray(P_t, dtype=np.float64)[k] @ np.asarray(V_next, dtype=np.float64)


def stage_bids(V_next: np.ndarray, P_t: np.ndarray, s: int, storage) -> List[BidCurve]:
    """One curve per observed price state k (a Markov chain makes the continuation value
    depend on k; with independent prices all K curves coincide)."""
    K = np.asarray(P_t).shape[0]
    return [bid_curve(expectation_row(V_next, P_t, k), s, storage) for k in range(K)]


def monotone_envelope(levels: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Least non-decreasing majorant of the points (levels[k], q[k]) in price order:
    out[k] = max{q[k'] : levels[k'] <= levels[k]} (equal levels share their maximum)."""
    levels = np.asarray(levels, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    order = np.argsort(levels, kind="stable")
    run = np.maximum.accumulate(q[order])
    out = np.empty_like(q)
    out[order] = run
    # states at one price level offer the largest quantity of the group
    lv = levels[order]
    i = 0
    while i < lv.size:
        e = i
        while e + 1 < lv.size and lv[e + 1] == lv[i]:
            e += 1
        out[order[i:e + 1]] = run[e]
        i = e + 1
    return out


@dataclasses.dataclass
class MarkovBid:
    """The bid for one stage and incoming SoC under a Markov price chain."""
    levels: np.ndarray   # lam_t[k]
    q: np.ndarray        # quantity each state's own curve clears at its level
    j: np.ndarray        # next state of that quantity (the DP policy where unique)
    q_bid: np.ndarray    # monotone envelope: quantity offered at each level
    j_bid: np.ndarray    # next state reached when the bid clears at level k
    profit: np.ndarray   # realised lam_t[k] q_bid + U_k(q_bid) at each level
    value: np.ndarray    # max_p lam_t[k] p + U_k(p) (the DP value V_t[k][s])

    @property
    def monotone_already(self) -> bool:
        return bool(np.array_equal(self.q, self.q_bid))

    def schedule(self):
        """(price, quantity) steps of the submitted curve, ascending in price."""
        o = np.argsort(self.levels, kind="stable")
        return [(float(self.levels[k]), float(self.q_bid[k])) for k in o]


def markov_bid(V_next: np.ndarray, P_t: np.ndarray, lam_t: np.ndarray, s: int, storage) -> MarkovBid:
    """Per-state curves (Eq. (7)-(10)) cleared at their own levels, combined into one
    monotone bid by the price-sorted envelope."""
    lam_t = np.asarray(lam_t, dtype=np.float64)
    curves = stage_bids(V_next, P_t, s, storage)
    K = len(curves)
    q = np.empty(K)
    jq = np.empty(K, dtype=np.int64)
    value = np.empty(K)
    for k, bc in enumerate(curves):
        q[k], jq[k], value[k] = bc.clear(float(lam_t[k]))
    q_bid = monotone_envelope(lam_t, q)
    j_bid = np.empty(K, dtype=np.int64)
    profit = np.empty(K)
    for k, bc in enumerate(curves):
        i = int(np.flatnonzero(bc.p == q_bid[k])[0])   # every curve has the same quantity grid
        j_bid[k] = bc.j[i]
        profit[k] = lam_t[k] * bc.p[i] + bc.U[i]
    return MarkovBid(levels=lam_t, q=q, j=jq, q_bid=q_bid, j_bid=j_bid, profit=profit,
                     value=value)
