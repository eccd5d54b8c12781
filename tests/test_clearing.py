"""Paper-mode bids and market clearing (host, FP64) against the continuous arbitrage
formulations of Eq. (1) and Eq. (3a)-(3d) solved exactly (CPU).  Values come from the
NumPy Algorithm 1 oracle; the clearing code is the product's."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import alg1
from oracle import arbitrage as ar
from oracle import hull as hull_oracle
from paper_2511_15629_amd import clearing


def values(lam, S, delta, eta, p_bar):
    """V_hat [T+1, S] of the deterministic problem (R = 1) by Algorithm 1 in FP64."""
    g = clearing.paper_grid(S, delta, eta, p_bar)
    s_hat = np.arange(S, dtype=np.float64) * g.delta
    p_hat, _, _ = alg1.power_grid(g.p_bar, g.delta, g.eta)
    assert np.allclose(p_hat, g.p, rtol=0, atol=1e-12)
    lam = np.asarray(lam, dtype=np.float64)[:, None]
    return alg1.algorithm1(s_hat, p_hat, lam, np.ones_like(lam), g.eta), g


def test_lossless_on_grid_bidding_and_dp_equal_the_lp():
    # eta = 1 and p_bar a multiple of delta: every action lands on the grid, the LP is
    # totally unimodular with an optimum on the grid, so DP = bidding = LP = MILP.
    lam = wl.realized_prices(96, seed=3)
    V, g = values(lam, 17, 0.25, 1.0, 1.0)
    lp = ar.arbitrage(lam, s_bar=g.s_bar, p_bar=1.0, eta=1.0, s0=0.0, mode="lp")["profit"]
    ex = ar.arbitrage(lam, s_bar=g.s_bar, p_bar=1.0, eta=1.0, s0=0.0, mode="exact")["profit"]
    sim = clearing.simulate_bidding(V, lam, 0.0, g)
    scale = max(1.0, abs(lp))
    assert abs(ex - lp) <= 1e-7 * scale
    assert abs(V[0][0] - lp) <= 1e-7 * scale
    assert abs(sim["profit"] - lp) <= 1e-7 * scale


@pytest.mark.parametrize("delta,floor", [(0.1, 0.97), (0.02, 0.99)])
def test_bidding_dispatch_is_feasible_and_below_the_milp(delta, floor):
    lam = wl.realized_prices(72, seed=5)
    eta = float(np.float32(math.sqrt(0.85)))
    S = int(round(4.0 / delta)) + 1
    V, g = values(lam, S, delta, eta, 1.0)
    sim = clearing.simulate_bidding(V, lam, 0.0, g)
    ex = ar.arbitrage(lam, s_bar=g.s_bar, p_bar=1.0, eta=g.eta, s0=0.0, mode="exact")["profit"]
    p, s = sim["p"], sim["s"]
    assert np.all(np.abs(p) <= g.p_bar + 1e-12)
    assert np.all((s >= 0.0) & (s <= g.s_bar))
    assert np.allclose(np.diff(s), clearing.transition(p, g.eta), rtol=0, atol=1e-8)
    assert abs(sim["profit"] - float(np.asarray(lam, np.float64) @ p)) <= 1e-9 * abs(sim["profit"])
    assert sim["profit"] <= ex + 1e-6 * abs(ex)
    assert sim["profit"] >= floor * ex


def test_cleared_quantity_attains_the_support_and_bids_are_monotone():
    lam = wl.negative_prices(wl.realized_prices(48, seed=8))
    eta = float(np.float32(math.sqrt(0.85)))
    V, g = values(lam, 41, 0.1, eta, 1.0)
    s = g.s_bar
    rng = np.random.default_rng(0)
    for t in range(1, 49):
        b = clearing.bid(V[t], s, g)
        prices = [seg[2] for seg in b.segments()]
        assert all(y >= x - 1e-9 for x, y in zip(prices, prices[1:]))
        for price in [float(lam[t - 1])] + list(rng.uniform(-300, 300, 3)):
            q, nxt, _ = b.clear(price)
            i = int(np.flatnonzero(b.p == q)[0])
            best = hull_oracle.support(b.p, b.U, price)
            assert abs(price * q + b.U[i] - best) <= 1e-9 * max(1.0, abs(best))
        q, s, _ = b.clear(float(lam[t - 1]))


def test_negative_price_formulations():
    # Sec. V-B: all prices <= 0, start full.  The LP restriction cannot discharge, so it
    # earns exactly 0; the relaxation overlaps charge and discharge and overstates the MILP;
    # the DP's cleared bids are a feasible dispatch close to the MILP.
    lam = wl.negative_prices(wl.realized_prices(72, seed=12))
    assert float(np.max(lam)) == 0.0
    eta = float(np.float32(math.sqrt(0.85)))
    kw = dict(s_bar=4.0, p_bar=1.0, eta=eta, s0=4.0)
    ex = ar.arbitrage(lam, mode="exact", **kw)
    rx = ar.arbitrage(lam, mode="relax", **kw)
    rs = ar.arbitrage(lam, mode="restrict", **kw)
    assert rs["profit"] == pytest.approx(0.0, abs=1e-9)
    assert ex["overlap"] == 0.0 and rx["overlap"] > 0.0
    assert rx["profit"] > ex["profit"] > 0.0
    V, g = values(lam, 41, 0.1, eta, 1.0)
    sim = clearing.simulate_bidding(V, lam, g.s_bar, g)
    assert sim["profit"] <= ex["profit"] + 1e-6 * ex["profit"]
    assert sim["profit"] >= 0.97 * ex["profit"]


def test_milp_pins():
    # eta = 1: overlapping charge and discharge gains nothing, so all formulations but the
    # restriction coincide; the MILP never beats the relaxation; a single stage is closed form.
    lam = wl.realized_prices(48, seed=9)
    kw = dict(s_bar=3.0, p_bar=1.0, eta=1.0, s0=1.0)
    vals = {m: ar.arbitrage(lam, mode=m, **kw)["profit"] for m in ("exact", "relax", "lp")}
    assert max(vals.values()) - min(vals.values()) <= 1e-7 * max(1.0, abs(vals["lp"]))
    eta = 0.9
    one = ar.arbitrage([50.0], s_bar=4.0, p_bar=1.0, eta=eta, s0=0.5, mode="exact")
    assert one["profit"] == pytest.approx(50.0 * 0.5 * eta)       # sell all 0.5 MWh
    one = ar.arbitrage([-20.0], s_bar=4.0, p_bar=1.0, eta=eta, s0=3.5, mode="exact")
    assert one["profit"] == pytest.approx(20.0 * 0.5 / eta)        # buy up to full
