"""Concave envelope of finitely many points by its definition.  TEST ONLY.

For points (x_i, y_i), the upper boundary of conv(hypograph) at x is the largest
value of a chord between two points whose x-range contains x (Eq. (9): hyp of the
convexified function = conv of hyp).  O(n^2) per query, written for clarity.
"""
from __future__ import annotations

import numpy as np


def envelope_at(xs, ys, x):
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    best = -np.inf
    n = xs.shape[0]
    for a in range(n):
        for b in range(n):
            xa, xb = xs[a], xs[b]
            if xa <= x <= xb:
                if xb == xa:
                    v = max(ys[a], ys[b])
                else:
                    w = (x - xa) / (xb - xa)
                    v = (1.0 - w) * ys[a] + w * ys[b]
                best = max(best, v)
    return best


def support(xs, ys, price):
    """max_x price * x + U(x) over the points (equal for U and its envelope)."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    return float(np.max(price * xs + ys))
