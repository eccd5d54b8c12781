"""Properties of the GPU solve that hold at any size, checked at the full five-minute day
shape (T = 288, K = 100, S = 1001, moves -250..250), where the oracle is too slow to
re-derive every output.

* Homogeneity in the prices: with no throughput or start cost, the payoff of Eq. (1) and
  the recursion of Eq. (5)-(6) are positively homogeneous in (lam, V).  Doubling lam is
  exact in binary floating point (every product, sum, maximum and normalisation offset
  doubles exactly), so the values double bit for bit and the policies are unchanged.
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
