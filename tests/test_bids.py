"""Host bid curves (Eq. (7)-(10)) against the definition of the concave envelope and the
oracle's DP values and policies (CPU)."""
import numpy as np
import pytest

import oracle
from oracle import hull as hull_oracle
import workloads as wl
from paper_2511_15629_amd import bids


def _instance(seed, c_start=0.0, lam_lo=-20.0):
    return wl.random_small(seed, 6, 3, 30, 6, 7, c_start=c_start, c_deg=1.0, lam_lo=lam_lo)


@pytest.mark.parametrize("seed,c_start,lam_lo", [(1, 0.0, -20.0), (2, 4.0, -20.0), (3, 0.0, -150.0)])
def test_hull_is_the_concave_envelope(seed, c_start, lam_lo):
    inst = _instance(seed, c_start, lam_lo)
    out = oracle.solve(inst.storage, inst.lam, inst.P)
    for t in (1, 3, 6):
        for s in (0, 7, 29):
            for k in range(3):
                w = bids.expectation_row(out["V"][t], inst.P[t - 1], k)
                bc = bids.bid_curve(w, s, inst.storage)
                for x in bc.p:
                    env = hull_oracle.envelope_at(bc.p, bc.U, x)
                    assert abs(bc.envelope(x) - env) <= 1e-9 * max(1.0, abs(env))


def test_bid_prices_are_monotone_and_support_is_preserved():
    inst = _instance(4, c_start=3.0, lam_lo=-100.0)
    out = oracle.solve(inst.storage, inst.lam, inst.P)
    rng = np.random.default_rng(0)
    for t in range(1, inst.T + 1):
        for s in range(0, 30, 5):
            w = bids.expectation_row(out["V"][t], inst.P[t - 1], 0)
            bc = bids.bid_curve(w, s, inst.storage)
            prices = [seg[2] for seg in bc.segments()]
            assert all(b >= a - 1e-9 for a, b in zip(prices, prices[1:]))
            for lam in rng.uniform(-200, 200, 5):
                _, _, prof = bc.clear(lam)
                assert abs(prof - hull_oracle.support(bc.p, bc.U, lam)) <= 1e-9 * max(1.0, abs(prof))


def test_cleared_quantity_reproduces_dp_value_and_policy():
    # At the realised price lam_t[k] the cleared profit equals V_t[k][s]; where the argmax
    # is unique and lies on the hull the cleared move is the DP policy.
    inst = _instance(5, c_start=0.0)
    out = oracle.solve(inst.storage, inst.lam, inst.P)
    agree = 0
    for t in range(1, inst.T + 1):
        for k in range(inst.K):
            for s in range(inst.storage.S):
                w = bids.expectation_row(out["V"][t], inst.P[t - 1], k)
                bc = bids.bid_curve(w, s, inst.storage)
                _, j, prof = bc.clear(float(inst.lam[t - 1, k]))
                assert abs(prof - out["V"][t - 1][k, s]) <= 1e-9 * max(1.0, abs(prof))
                agree += int(j == out["policy"][t - 1][k, s])
    assert agree >= 0.95 * inst.T * inst.K * inst.storage.S


def test_start_cost_makes_the_envelope_bridge_the_idle_point():
    # With a start cost the idle move sits above its neighbours' chord by c_start; the
    # envelope keeps it (the bid has a dead band) and drops nothing else when W is linear.
    st = wl.Storage(S=21, w_up=5, w_down=5, delta=0.1, eta_c=1.0, eta_d=1.0, c_start=2.0)
    w = np.linspace(0.0, 10.0, 21)
    bc = bids.bid_curve(w, 10, st)
    assert 10 in bc.j[bc.hull]
    segs = bc.segments()
    assert any(a < 0.0 < b or b == 0.0 or a == 0.0 for a, b, _ in segs)


def test_monotone_envelope_is_the_least_nondecreasing_majorant():
    # Definition pin by enumeration: among all non-decreasing integer schedules on 0..4 that
    # lie on or above q at every level (in price order), the pointwise minimum is the one
    # returned (ties in price share one offer).
    import itertools
    rng = np.random.default_rng(9)
    for _ in range(40):
        K = int(rng.integers(1, 6))
        levels = rng.choice([-5.0, 0.0, 3.0, 7.5, 20.0], size=K)
        q = rng.integers(0, 5, size=K).astype(np.float64)
        o = np.argsort(levels, kind="stable")
        best = None
        for cand in itertools.product(range(5), repeat=K):
            c = np.array(cand, dtype=np.float64)
            ok = np.all(c >= q)
            ok &= all(c[o[i]] <= c[o[i + 1]] for i in range(K - 1))
            ok &= all(c[a] == c[b] for a in range(K) for b in range(K) if levels[a] == levels[b])
            if ok:
                best = c if best is None else np.minimum(best, c)
        np.testing.assert_array_equal(bids.monotone_envelope(levels, q), best)


def test_independent_prices_bid_is_monotone_and_clears_the_dp_value():
    # With every row of P_t equal (stagewise independence, the paper's setting) all states
    # share one concave U~, so the per-state quantities are already non-decreasing in price
    # and the combined bid clears exactly the DP value at every level.
    rng = np.random.default_rng(11)
    T, K, S = 6, 5, 30
    lam = wl.f32(rng.uniform(-40, 90, size=(T, K)))
    rows = wl.quantize_rows(rng.dirichlet(np.ones(K), size=T))
    P = np.repeat(rows[:, None, :], K, axis=1)
    st = wl.Storage(S=S, w_up=6, w_down=7, delta=0.25, eta_c=0.9, eta_d=0.9, c_deg=1.0).as_f32()
    out = oracle.solve(st, lam, P)
    for t in range(1, T + 1):
        for s in range(S):
            mb = bids.markov_bid(out["V"][t], P[t - 1], lam[t - 1], s, st)
            assert mb.monotone_already
            np.testing.assert_allclose(mb.profit, out["V"][t - 1][:, s], rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed,c_start", [(6, 0.0), (7, 3.0)])
def test_markov_bid_is_monotone_and_never_beats_the_dp(seed, c_start):
    inst = wl.random_small(seed, 6, 6, 30, 6, 7, c_start=c_start, lam_lo=-80.0)
    out = oracle.solve(inst.storage, inst.lam, inst.P)
    n_mono = 0
    for t in range(1, inst.T + 1):
        for s in range(inst.storage.S):
            mb = bids.markov_bid(out["V"][t], inst.P[t - 1], inst.lam[t - 1], s, inst.storage)
            sched = mb.schedule()
            assert all(b[1] >= a[1] for a, b in zip(sched, sched[1:]))
            assert np.all(mb.q_bid >= mb.q)
            np.testing.assert_allclose(mb.value, out["V"][t - 1][:, s], rtol=0, atol=1e-9)
            assert np.all(mb.profit <= mb.value + 1e-9)
            if mb.monotone_already:
                n_mono += 1
                np.testing.assert_allclose(mb.profit, mb.value, rtol=0, atol=1e-9)
    print(f"per-state quantities already monotone in price at {n_mono} of "
          f"{inst.T * inst.storage.S} (t, s)")
