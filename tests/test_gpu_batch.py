"""GPU tests of the batched solve (dp_batch_* through the C ABI).

The batched path must give bitwise the same V_1 and policies as one dp_solve per
instance (the looped path), whatever tile classes the plan picks, and match the oracle.
"""
import dataclasses
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from parity import RTOL, _mismatch, value_error

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_15629_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def small_batch():
    specs = [
        (1, 6, 3, 50, 5, 7, {}), (2, 6, 17, 300, 30, 45, {}), (3, 9, 20, 700, 60, 90, dict(c_start=2.0)),
        (4, 4, 5, 129, 128, 128, {}), (5, 6, 1, 10, 2, 3, {}), (6, 12, 8, 257, 3, 1, {}),
        (7, 6, 33, 600, 250, 250, dict(lam_lo=-150.0)), (8, 5, 12, 1001, 14, 18, dict(eta=0.86)),
        (9, 6, 2, 2, 1, 1, {}), (10, 7, 64, 512, 0, 0, {}),
        (11, 1, 9, 150, 12, 9, {}), (12, 2, 40, 90, 30, 30, dict(c_start=1.0)),   # T = 1, 2 beside T = 12
    ]
    return [wl.random_small(sd, T, K, S, wu, wd, **kw) for (sd, T, K, S, wu, wd, kw) in specs]


def run_batch(dp, plan, insts, looped=False, lam_override=None, graph=True):
    lams = [dev(i.lam if lam_override is None else lam_override[n]) for n, i in enumerate(insts)]
    Ps = [dev(i.P) for i in insts]
    V1 = [torch.full((i.K, i.storage.S), float("nan"), device="cuda") for i in insts]
    pol = [torch.full((i.T, i.K, i.storage.S), -1, dtype=torch.int16, device="cuda") for i in insts]
    plan.solve(lams, Ps, V1, pol, looped=looped, graph=graph)
    torch.cuda.synchronize()
    return V1, pol


def test_batched_equals_looped_bitwise_and_matches_oracle(dp):
    insts = small_batch()
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts])
    print(plan.describe())
    Vb, pb = run_batch(dp, plan, insts)
    Vl, pl = run_batch(dp, plan, insts, looped=True)
    for n, inst in enumerate(insts):
        assert torch.equal(Vb[n], Vl[n]), inst.name
        assert torch.equal(pb[n], pl[n]), inst.name
        ref = oracle.solve(inst.storage, inst.lam, inst.P)
        assert value_error(Vb[n].cpu().numpy(), ref["V"][0]) <= RTOL, inst.name
        pol = pb[n].cpu().numpy()
        for t in range(1, inst.T + 1):
            if not np.array_equal(pol[t - 1], ref["policy"][t - 1]):
                _mismatch(inst.storage, inst.lam[t - 1], inst.P[t - 1], ref["V"][t],
                          ref["V"][t - 1], pol[t - 1], ref["policy"][t - 1],
                          f"{inst.name} stage {t}")
    plan.close()


def test_rows_off_the_simplex_batched_equals_looped_and_oracle(dp):
    insts = [dataclasses.replace(i, P=wl.unnormalised_rows(i.P, 2e-6, seed=n))
             for n, i in enumerate(small_batch()[:8])]
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts])
    Vb, pb = run_batch(dp, plan, insts)
    Vl, pl = run_batch(dp, plan, insts, looped=True)
    for n, inst in enumerate(insts):
        assert torch.equal(Vb[n], Vl[n]) and torch.equal(pb[n], pl[n]), inst.name
        ref = oracle.solve(inst.storage, inst.lam, inst.P)
        assert value_error(Vb[n].cpu().numpy(), ref["V"][0]) <= RTOL, inst.name
    plan.close()


def test_replay_with_new_pointers_and_data(dp):
    insts = small_batch()[:5]
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts])
    run_batch(dp, plan, insts)
    rng = np.random.default_rng(7)
    lam2 = [wl.f32(i.lam.astype(np.float64) + rng.normal(0, 10, i.lam.shape)) for i in insts]
    Vb, pb = run_batch(dp, plan, insts, lam_override=lam2)
    for n, inst in enumerate(insts):
        out = dp.solve(dev(lam2[n]), dev(inst.P), inst.storage, store_all=False, policy=True)
        torch.cuda.synchronize()
        assert torch.equal(Vb[n], out["V"]) and torch.equal(pb[n], out["policy"])
    plan.close()


def test_eager_launches_equal_graph_replay(dp):
    # every expectation group (K <= 32, <= 64, <= 128, > 128) present, so all four branches
    # are forked and joined; the eager path issues the captured launches directly
    specs = [(31, 5, 7, 120, 6, 9, {}), (32, 4, 40, 300, 25, 20, {}), (33, 6, 90, 260, 40, 35, {}),
             (34, 3, 140, 200, 12, 10, dict(c_start=1.0)), (35, 5, 20, 700, 80, 60, {})]
    insts = [wl.random_small(sd, T, K, S, wu, wd, **kw) for (sd, T, K, S, wu, wd, kw) in specs]
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts])
    Vg, pg = run_batch(dp, plan, insts)
    for rep in range(2):
        Ve, pe = run_batch(dp, plan, insts, graph=False)
        for n, inst in enumerate(insts):
            assert torch.equal(Vg[n], Ve[n]) and torch.equal(pg[n], pe[n]), (inst.name, rep)
    Vl, pl = run_batch(dp, plan, insts, looped=True)
    for n, inst in enumerate(insts):
        assert torch.equal(Vg[n], Vl[n]) and torch.equal(pg[n], pl[n]), inst.name
    plan.close()


def test_large_chains_use_strips_and_equal_looped(dp):
    # K > 128 takes the 64-column strip expectation, K <= 128 the LDS panels; mixed in one plan
    specs = [(21, 4, 130, 300, 20, 25, {}), (22, 3, 200, 150, 9, 7, dict(c_start=1.0)),
             (23, 5, 100, 257, 40, 40, {}), (24, 4, 129, 64, 3, 5, {})]
    insts = [wl.random_small(sd, T, K, S, wu, wd, **kw) for (sd, T, K, S, wu, wd, kw) in specs]
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts])
    text = plan.describe()
    assert "strips" in text and " 0 strips" not in text, text
    Vb, pb = run_batch(dp, plan, insts)
    Vl, pl = run_batch(dp, plan, insts, looped=True)
    for n, inst in enumerate(insts):
        assert torch.equal(Vb[n], Vl[n]) and torch.equal(pb[n], pl[n]), inst.name
        ref = oracle.solve(inst.storage, inst.lam, inst.P, keep_all=False, want_policy=False)
        assert value_error(Vb[n].cpu().numpy(), ref["V1"]) <= RTOL, inst.name
    plan.close()


def test_repeated_replays_match_eager_each_time(dp):
    # the captured graph is replayed several times, alternating two price sets, with the
    # program's own eager work and synchronisations between replays; every replay must
    # equal the eager solve of its data
    insts = small_batch()[:6]
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts])
    rng = np.random.default_rng(11)
    sets = [[i.lam for i in insts],
            [wl.f32(i.lam.astype(np.float64) + rng.normal(0, 15, i.lam.shape)) for i in insts]]
    eager = []
    for lams in sets:
        outs = []
        for n, inst in enumerate(insts):
            o = dp.solve(dev(lams[n]), dev(inst.P), inst.storage, store_all=False, policy=True)
            outs.append((o["V"].clone(), o["policy"].clone()))
        torch.cuda.synchronize()
        eager.append(outs)
    for rep in range(4):
        which = rep % 2
        Vb, pb = run_batch(dp, plan, insts, lam_override=sets[which])
        junk = torch.randn(1 << 16, device="cuda").sum()        # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for n, inst in enumerate(insts):
            assert torch.equal(Vb[n], eager[which][n][0]), (rep, inst.name)
            assert torch.equal(pb[n], eager[which][n][1]), (rep, inst.name)
    plan.close()


def test_autotuned_plan_is_bitwise_equal_and_cache_is_reused(dp, tmp_path):
    insts = small_batch()
    cache = str(tmp_path / "tune.txt")
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts], tune_cache=cache)
    text = plan.describe()
    print(text)
    assert "autotuned" in text and os.path.exists(cache)
    Vb, pb = run_batch(dp, plan, insts)
    plan.close()
    lines = open(cache).read().splitlines()
    plan2 = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts], tune_cache=cache)
    assert "autotuned" not in plan2.describe()
    assert open(cache).read().splitlines() == lines
    Vl, pl = run_batch(dp, plan2, insts, looped=True)
    for n in range(len(insts)):
        assert torch.equal(Vb[n], Vl[n]) and torch.equal(pb[n], pl[n])
    plan2.close()


def test_fleet_of_512_batched_equals_looped(dp):
    """The 512-battery fleet: batched V_1 and all policies bitwise equal to the looped
    solves, and values and policies of instances from every K class (the smallest and
    largest, and a random pick) against the oracle, stage by stage under the near-tie rule."""
    insts = wl.fleet_5min()
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts])
    print(plan.describe())
    cache = {}
    lams = [dev(i.lam) for i in insts]
    Ps = []
    for i in insts:
        if id(i.P) not in cache:
            cache[id(i.P)] = dev(i.P)
        Ps.append(cache[id(i.P)])
    Vb = [torch.empty(i.K, i.storage.S, device="cuda") for i in insts]
    pb = [torch.empty(i.T, i.K, i.storage.S, dtype=torch.int16, device="cuda") for i in insts]
    plan.solve(lams, Ps, Vb, pb)
    Vl = [torch.empty(i.K, i.storage.S, device="cuda") for i in insts]
    pl = [torch.empty(i.T, i.K, i.storage.S, dtype=torch.int16, device="cuda") for i in insts]
    plan.solve(lams, Ps, Vl, pl, looped=True)
    torch.cuda.synchronize()
    for n in range(len(insts)):
        assert torch.equal(Vb[n], Vl[n]) and torch.equal(pb[n], pl[n]), insts[n].name
    del Vl, pl
    by_size = sorted(range(len(insts)), key=lambda n: insts[n].candidates())
    rng = np.random.default_rng(4)
    picks = by_size[:2] + by_size[-2:]
    for K in (20, 50, 100):
        picks.append(int(rng.choice([n for n in range(len(insts)) if insts[n].K == K])))
    total = 0
    for n in picks:
        inst = insts[n]
        ref = oracle.solve(inst.storage, inst.lam, inst.P)
        v1 = Vb[n].cpu().numpy()
        assert value_error(v1, ref["V"][0]) <= RTOL, inst.name
        pol = pb[n].cpu().numpy()
        for t in range(1, inst.T + 1):          # the batch returns V_1 and every policy
            total += _mismatch(inst.storage, inst.lam[t - 1], inst.P[t - 1], ref["V"][t],
                               ref["V"][t - 1], pol[t - 1], ref["policy"][t - 1],
                               f"{inst.name} stage {t}")
    print(f"fleet: {len(picks)} instances against the oracle, accepted near-ties {total}")
    plan.close()


def test_plan_rejects_flags(dp):
    inst = wl.random_small(1, 3, 2, 10, 1, 1)
    from paper_2511_15629_amd import _lib
    import ctypes
    pb = _lib.make_problem(3, 2, inst.storage, _lib.DP_STORE_V_ALL)
    arr = (_lib.Problem * 1)(pb)
    h = ctypes.c_void_p()
    rc = _lib.lib().dp_batch_plan_create(ctypes.byref(h), 1, arr, None, None)
    assert rc == -1 and not h.value
