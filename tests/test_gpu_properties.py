"""Properties of the GPU solves that hold at any size, checked at full sizes where the
oracle is too slow to re-derive every output: the five-minute day (T = 288, K = 100,
S = 1001, moves -250..250), a Table 3 shape of the paper mode (T = 8784, R = 200, S = 2001,
P = 203) and the 512-battery fleet.

* Homogeneity in the prices: with no throughput or start cost, the payoff of Eq. (1) and
  the recursion of Eq. (5)-(6) are positively homogeneous in (lam, V).  Doubling lam is
  exact in binary floating point (every product, sum, maximum and normalisation offset
  doubles exactly), so the values double bit for bit and the policies are unchanged.  The
  same holds for the paper mode (payoff lam p, interpolated endpoints) and for the batch.
* Relabelling the price states permutes the value rows (the expectation sums in another
  order, so within the FP32 tolerance).
* A constant terminal value c adds c to every V_t, since every row of P_t sums to 1
  (within the FP32 tolerance: the row sums are exact, the products are rounded).
"""
import dataclasses

import numpy as np
import pytest

import workloads as wl
from parity import RTOL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15629_amd as m
    return m


@pytest.fixture(scope="module")
def day():
    return wl.day_5min()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def normwise(a, b):
    """max |a - b| / max |b| per stage, worst stage."""
    a = a.double()
    b = b.double()
    err = (a - b).abs().flatten(1).amax(1)
    scale = b.abs().flatten(1).amax(1).clamp_min(1e-30)
    return float((err / scale).max())


def test_doubling_prices_doubles_values_bitwise(dp, day):
    st = dataclasses.replace(day.storage, c_deg=0.0, c_start=0.0)
    a = dp.solve(dev(day.lam), dev(day.P), st, store_all=True)
    b = dp.solve(dev(2.0 * day.lam), dev(day.P), st, store_all=True)
    torch.cuda.synchronize()
    assert torch.equal(b["V"], 2.0 * a["V"])
    assert torch.equal(b["policy"], a["policy"])


def test_relabelled_price_states_permute_values(dp, day):
    perm = np.random.default_rng(5).permutation(day.K)
    lam_p = day.lam[:, perm]
    P_p = day.P[:, perm][:, :, perm]
    a = dp.solve(dev(day.lam), dev(day.P), day.storage, store_all=True)
    b = dp.solve(dev(lam_p), dev(P_p), day.storage, store_all=True)
    torch.cuda.synchronize()
    err = normwise(b["V"], a["V"][:, torch.from_numpy(perm).cuda()])
    print(f"relabelled states: normwise value error {err:.2e}")
    assert err <= RTOL


def test_constant_terminal_value_shifts_every_stage(dp, day):
    c = 37.5
    S = day.storage.S
    a = dp.solve(dev(day.lam), dev(day.P), day.storage, store_all=True)
    v_term = torch.full((day.K, S), c, device="cuda")
    b = dp.solve(dev(day.lam), dev(day.P), day.storage, v_term, store_all=True)
    torch.cuda.synchronize()
    err = normwise(b["V"][:-1], a["V"][:-1] + c)
    print(f"terminal shift {c}: normwise value error {err:.2e}")
    assert err <= RTOL
    assert torch.equal(b["V"][-1], v_term)


def test_paper_mode_doubling_prices_doubles_values_bitwise(dp):
    # the Table 3 shape S = 2001, P = 203 (20 h, delta = 0.01), full year, R = 200
    inst = wl.table3_instance(20, 0.01)
    lam, prob = dev(inst.lam), dev(inst.prob)
    kw = dict(store_all=True, policy=True)
    a = dp.solve_independent(lam, prob, inst.S, inst.delta, inst.eta, inst.p_bar, **kw)
    b = dp.solve_independent(2.0 * lam, prob, inst.S, inst.delta, inst.eta, inst.p_bar, **kw)
    torch.cuda.synchronize()
    assert torch.equal(b["V"], 2.0 * a["V"])
    assert torch.equal(b["policy"], a["policy"])


def test_fleet_doubling_prices_doubles_values_bitwise(dp):
    insts = wl.fleet_5min()
    sts = [dataclasses.replace(i.storage, c_deg=0.0, c_start=0.0) for i in insts]
    plan = dp.BatchPlan([(i.T, i.K, st) for i, st in zip(insts, sts)])
    Ps = {}
    for i in insts:
        if id(i.P) not in Ps:
            Ps[id(i.P)] = dev(i.P)
    P = [Ps[id(i.P)] for i in insts]
    out = []
    for scale in (1.0, 2.0):
        lams = [dev(scale * i.lam) for i in insts]
        V1 = [torch.empty(i.K, i.storage.S, device="cuda") for i in insts]
        pol = [torch.empty(i.T, i.K, i.storage.S, dtype=torch.int16, device="cuda") for i in insts]
        plan.solve(lams, P, V1, pol)
        torch.cuda.synchronize()
        out.append((V1, pol))
    plan.close()
    for n, inst in enumerate(insts):
        assert torch.equal(out[1][0][n], 2.0 * out[0][0][n]), inst.name
        assert torch.equal(out[1][1][n], out[0][1][n]), inst.name
