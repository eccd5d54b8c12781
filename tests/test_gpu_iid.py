"""GPU parity of the stagewise-independent solve on the paper's power grid (dp_solve_iid)
against Algorithm 1 written out in NumPy FP64 (oracle/alg1.py)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import alg1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
RTOL = 1e-5


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15629_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def grid(S, delta, eta, p_bar):
    s_hat = np.arange(S, dtype=np.float64) * float(np.float32(delta))
    p_hat, n_c, n_d = alg1.power_grid(float(np.float32(p_bar)), float(np.float32(delta)),
                                      float(np.float32(eta)))
    return s_hat, p_hat, n_c, n_d


def normwise(a, b):
    return float(np.max(np.abs(a.astype(np.float64) - b))) / max(float(np.max(np.abs(b))), 1e-30)


def check_policy(pol_gpu, Q_all, v_or):
    """Mismatches accepted only where the GPU's action is within the tolerance of the max."""
    pol_or = alg1.policy_index(Q_all)                   # [S, R]
    mism = np.argwhere(pol_gpu.T != pol_or)             # pol_gpu is [R, S]
    tol = RTOL * max(float(np.max(np.abs(v_or))), 1e-30)
    qmax = Q_all.max(axis=1)
    for s, r in mism:
        q = Q_all[s, int(pol_gpu[r, s]), r]
        assert np.isfinite(q) and q >= qmax[s, r] - tol, (s, r, q, qmax[s, r])
    return int(mism.shape[0])


CASES = [
    dict(T=6, R=5, S=21, delta=0.1, eta=0.9, p_bar=0.47),
    dict(T=9, R=17, S=101, delta=0.04, eta=math.sqrt(0.85), p_bar=1.0),
    dict(T=5, R=3, S=7, delta=0.5, eta=0.8, p_bar=2.0),        # power range beyond the storage
    dict(T=4, R=64, S=401, delta=0.01, eta=math.sqrt(0.85), p_bar=1.0),   # P = 203
    dict(T=7, R=2, S=33, delta=0.25, eta=1.0, p_bar=1.0),      # integral endpoints (b = 0)
    dict(T=1, R=1, S=2, delta=0.5, eta=0.9, p_bar=0.3),        # one stage, one sample, two levels
    dict(T=3, R=300, S=9, delta=0.2, eta=0.95, p_bar=0.1),     # power below one grid step
]


@pytest.mark.parametrize("c", CASES, ids=lambda c: f"S{c['S']}_R{c['R']}_d{c['delta']}")
def test_small_cases_match_algorithm1(dp, c):
    lam, prob = wl.iid_prices(c["T"], c["R"], seed=c["S"])
    s_hat, p_hat, n_c, n_d = grid(c["S"], c["delta"], c["eta"], c["p_bar"])
    P, gc, gd = dp.power_grid_size(c["S"], c["delta"], c["eta"], c["p_bar"])
    assert (P, gc, gd) == (p_hat.shape[0], n_c, n_d)
    out = dp.solve_independent(dev(lam), dev(prob), c["S"], c["delta"], c["eta"], c["p_bar"],
                               store_all=True, policy=True)
    torch.cuda.synchronize()
    V = out["V"].cpu().numpy()
    pol = out["policy"].cpu().numpy()
    pre = alg1.precompute(s_hat, p_hat, float(np.float32(c["eta"])))
    Vo = np.zeros(c["S"])
    for t in range(c["T"], 0, -1):
        v_prev, Q_all = alg1.stage(pre, p_hat, lam[t - 1], prob[t - 1], Vo)
        assert normwise(V[t - 1], v_prev) <= RTOL, t
        check_policy(pol[t - 1], Q_all, v_prev)
        Vo = v_prev
    ref = alg1.algorithm1(s_hat, p_hat, lam, prob, float(np.float32(c["eta"])))
    assert normwise(V[0], ref[0]) <= RTOL


def test_table3_smallest_full_year_matches_algorithm1(dp):
    """4 h battery, delta = 0.1 (S = 41, P = 22), 8784 hourly stages, 200 samples."""
    inst = wl.table3_instance(4, 0.1)
    out = dp.solve_independent(dev(inst.lam), dev(inst.prob), inst.S, inst.delta, inst.eta,
                               inst.p_bar, store_all=True)
    torch.cuda.synchronize()
    V = out["V"].cpu().numpy()
    s_hat, p_hat, _, _ = grid(inst.S, inst.delta, inst.eta, inst.p_bar)
    ref = alg1.algorithm1(s_hat, p_hat, inst.lam, inst.prob, inst.eta)
    for t in (0, 1, 100, 4392, 8783, 8784):
        assert normwise(V[t], ref[t]) <= RTOL, t


@pytest.mark.parametrize("hours,delta", [(100, 0.01), (20, 0.01)])
def test_table3_large_sampled_stages(dp, hours, delta):
    """S = 10001 / 2001, P = 203: stages re-derived by Algorithm 1 from the GPU's V_t."""
    inst = wl.table3_instance(hours, delta)
    out = dp.solve_independent(dev(inst.lam), dev(inst.prob), inst.S, inst.delta, inst.eta,
                               inst.p_bar, store_all=True, policy=True)
    torch.cuda.synchronize()
    s_hat, p_hat, _, _ = grid(inst.S, inst.delta, inst.eta, inst.p_bar)
    pre = alg1.precompute(s_hat, p_hat, inst.eta)
    rows = np.unique(np.linspace(0, inst.S - 1, 41).astype(np.int64))
    for t in (inst.T, 5000, 1):
        v_next = out["V"][t].cpu().numpy().astype(np.float64)
        v_gpu = out["V"][t - 1].cpu().numpy()
        v_or, Q_all = alg1.stage(pre, p_hat, inst.lam[t - 1], inst.prob[t - 1], v_next, rows=rows)
        scale = max(float(np.max(np.abs(v_or))), float(np.max(np.abs(v_gpu))), 1e-30)
        assert float(np.max(np.abs(v_gpu[rows] - v_or))) <= RTOL * scale, t
        pol = out["policy"][t - 1].cpu().numpy()[:, rows]
        check_policy(pol, Q_all, v_or)
    del out
    torch.cuda.empty_cache()


def test_maximum_grid_sampled_stages(dp):
    """S = 32767 levels (the int16 limit) with P = 2013 actions and 3 samples."""
    T, R, S, delta, eta, p_bar = 3, 3, 32767, 0.001, 0.9, 1.0
    lam, prob = wl.iid_prices(T, R, seed=77)
    out = dp.solve_independent(dev(lam), dev(prob), S, delta, eta, p_bar, store_all=True,
                               policy=True)
    torch.cuda.synchronize()
    s_hat, p_hat, _, _ = grid(S, delta, eta, p_bar)
    assert p_hat.shape[0] == 2013
    pre = alg1.precompute(s_hat, p_hat, float(np.float32(eta)))
    rows = np.unique(np.concatenate([np.arange(0, 40), np.linspace(0, S - 1, 61).astype(np.int64),
                                     np.arange(S - 40, S)]))
    for t in range(T, 0, -1):
        v_next = out["V"][t].cpu().numpy().astype(np.float64)
        v_gpu = out["V"][t - 1].cpu().numpy()
        v_or, Q_all = alg1.stage(pre, p_hat, lam[t - 1], prob[t - 1], v_next, rows=rows)
        scale = max(float(np.max(np.abs(v_or))), float(np.max(np.abs(v_gpu))), 1e-30)
        assert float(np.max(np.abs(v_gpu[rows] - v_or))) <= RTOL * scale, t
        check_policy(out["policy"][t - 1].cpu().numpy()[:, rows], Q_all, v_or)


def test_probabilities_off_the_simplex_long_horizon(dp):
    """Sample probabilities summing to 1 only within 2e-6 over 2000 stages: the offset
    carried between stages is weighted by the probability sum, as the expectation is."""
    T, R, S, delta, eta, p_bar = 2000, 20, 101, 0.04, math.sqrt(0.85), 1.0
    lam, prob = wl.iid_prices(T, R, seed=5)
    prob = wl.unnormalised_rows(prob, 2e-6, seed=5)
    assert np.abs(prob.astype(np.float64).sum(-1) - 1.0).max() > 1e-6
    s_hat, p_hat, _, _ = grid(S, delta, eta, p_bar)
    out = dp.solve_independent(dev(lam), dev(prob), S, delta, eta, p_bar, store_all=True)
    torch.cuda.synchronize()
    V = out["V"].cpu().numpy()
    pre = alg1.precompute(s_hat, p_hat, float(np.float32(eta)))
    Vo = np.zeros(S)
    for t in range(T, 0, -1):
        Vo, _ = alg1.stage(pre, p_hat, lam[t - 1], prob[t - 1], Vo)
        assert normwise(V[t - 1], Vo) <= RTOL, t
