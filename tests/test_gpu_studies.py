"""Deterministic studies of Sec. V on synthetic prices, with the DP solved on the GPU
(paper mode, R = 1) and the continuous formulations solved exactly by the oracle.

* Table 1 analog: a year of hourly perfect-foresight prices, 4 h battery, delta refined
  0.1 -> 0.01 (P = 22 -> 203); DP value and cleared bids against the LP upper bound.
* Table 2 analog: 72 h of all-negative prices starting full; MILP, LP relaxation and LP
  restriction against the DP value and its cleared bids.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import alg1
from oracle import arbitrage as ar

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ETA = float(np.float32(math.sqrt(0.85)))


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15629_amd as m
    return m


def gpu_values(dp, lam, S, delta):
    lam2 = torch.from_numpy(np.ascontiguousarray(lam[:, None])).cuda()
    prob = torch.ones_like(lam2)
    out = dp.solve_independent(lam2, prob, S, delta, ETA, 1.0, store_all=True)
    torch.cuda.synchronize()
    return out["V"].cpu().numpy().astype(np.float64)


def test_delta_refinement_year(dp):
    from paper_2511_15629_amd import clearing
    lam = wl.realized_prices(8784, seed=11)
    lp = ar.arbitrage(lam, s_bar=4.0, p_bar=1.0, eta=ETA, s0=0.0, mode="lp")["profit"]
    rows = []
    for delta in (0.1, 0.05, 0.02, 0.01):
        S = int(round(4.0 / delta)) + 1
        V = gpu_values(dp, lam, S, delta)
        g = clearing.paper_grid(S, delta, ETA, 1.0)
        if delta == 0.1:     # the whole GPU value vector against Algorithm 1 in FP64
            ref = alg1.algorithm1(np.arange(S) * g.delta, g.p, lam.astype(np.float64)[:, None],
                                  np.ones((8784, 1)), g.eta)
            assert np.max(np.abs(V[0] - ref[0])) <= 1e-5 * np.max(np.abs(ref[0]))
        sim = clearing.simulate_bidding(V, lam, 0.0, g)
        rows.append((delta, g.p.shape[0], V[0][0], sim["profit"]))
    print("\nTable 1 analog (synthetic year, 4 h, eta = sqrt(0.85)): LP %.2f" % lp)
    for delta, P, q, b in rows:
        print(f"  delta {delta:5.2f} P {P:4d}  DP {q:10.2f} ({(q - lp) / lp:+.4%})"
              f"  bidding {b:10.2f} ({(b - lp) / lp:+.4%})")
    for delta, P, q, b in rows:
        assert b <= lp + 1e-6 * abs(lp)               # a feasible dispatch
        assert q <= lp + 1e-5 * abs(lp)               # the DP is a restriction (FP32 slack)
        assert q >= 0.98 * lp and b >= 0.98 * lp
    gaps = [lp - q for _, _, q, _ in rows]
    assert gaps[-1] < gaps[0]                          # refining delta closes the gap


def test_negative_prices_72h(dp):
    from paper_2511_15629_amd import clearing
    lam = wl.negative_prices(wl.realized_prices(72, seed=12))
    kw = dict(s_bar=4.0, p_bar=1.0, eta=ETA, s0=4.0)
    res = {m: ar.arbitrage(lam, mode=m, **kw) for m in ("exact", "relax", "restrict")}
    ex = res["exact"]["profit"]
    S, delta = 401, 0.01
    V = gpu_values(dp, lam, S, delta)
    g = clearing.paper_grid(S, delta, ETA, 1.0)
    sim = clearing.simulate_bidding(V, lam, g.s_bar, g)
    q = V[0][S - 1]
    print("\nTable 2 analog (synthetic 72 h, all prices <= 0, start full):")
    for m, r in res.items():
        print(f"  {m:9s} {r['profit']:9.3f} ({(r['profit'] - ex) / ex:+.2%})  overlap {r['overlap']:.0%}")
    print(f"  DP        {q:9.3f} ({(q - ex) / ex:+.2%})\n  DP bids   {sim['profit']:9.3f}"
          f" ({(sim['profit'] - ex) / ex:+.2%})")
    assert res["restrict"]["profit"] == pytest.approx(0.0, abs=1e-9)
    assert res["relax"]["profit"] > ex and res["relax"]["overlap"] > 0.0
    assert sim["profit"] <= ex + 1e-6 * ex
    assert sim["profit"] >= 0.99 * ex and q >= 0.99 * ex
