"""GPU parity of the backward induction (dp_solve through the C ABI) against the oracle."""
import dataclasses
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from parity import RTOL, check_solve, check_stage, value_error

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


def gpu_solve(dp, inst, v_term=None, **kw):
    out = dp.solve(dev(inst.lam), dev(inst.P), inst.storage,
                   None if v_term is None else dev(v_term.astype(np.float32)), **kw)
    torch.cuda.synchronize()
    return out


def full_parity(dp, inst, v_term=None, threads=0):
    out = gpu_solve(dp, inst, v_term, store_all=True)
    V = out["V"].cpu().numpy()
    pol = out["policy"].cpu().numpy()
    ref = oracle.solve(inst.storage, inst.lam, inst.P,
                       None if v_term is None else v_term.astype(np.float32).astype(np.float64),
                       threads=threads)
    n = check_solve(inst.storage, inst.lam, inst.P, V, pol, ref, label=inst.name)
    return n, V, pol, ref


RAGGED = [
    dict(seed=1, T=5, K=3, S=7, wu=2, wd=3, c_start=1.0),
    dict(seed=2, T=6, K=17, S=600, wu=40, wd=70),
    dict(seed=3, T=4, K=33, S=1300, wu=300, wd=5, c_start=2.5),
    dict(seed=4, T=3, K=1, S=2, wu=1, wd=1),
    dict(seed=5, T=4, K=5, S=40, wu=0, wd=0),
    dict(seed=6, T=3, K=4, S=257, wu=256, wd=256, lam_lo=-150.0),
    dict(seed=7, T=5, K=64, S=512, wu=64, wd=64, c_deg=0.0),
    dict(seed=8, T=4, K=20, S=2001, wu=160, wd=190, eta=0.86),
    dict(seed=9, T=7, K=2, S=129, wu=1, wd=100),
    dict(seed=10, T=1, K=6, S=300, wu=20, wd=35, c_start=1.0),    # a single stage
    dict(seed=11, T=1, K=1, S=2, wu=1, wd=1),                     # the smallest problem
    # the direct maximum takes move ranges of up to 96 moves (idle included), the window
    # scans longer ones: the two sides of that boundary
    dict(seed=12, T=4, K=9, S=900, wu=50, wd=45, c_start=1.5),
    dict(seed=13, T=4, K=9, S=900, wu=50, wd=46, c_start=1.5),
]


@pytest.mark.parametrize("case", RAGGED, ids=lambda c: f"s{c['seed']}_K{c['K']}_S{c['S']}")
def test_ragged_shapes_match_oracle(dp, case):
    kw = dict(case)
    seed, T, K, S, wu, wd = (kw.pop(k) for k in ("seed", "T", "K", "S", "wu", "wd"))
    inst = wl.random_small(seed, T, K, S, wu, wd, **kw)
    v_term = None
    if seed % 3 == 0:
        v_term = np.random.default_rng(seed).uniform(-20, 20, size=(K, S))
    n, V, pol, ref = full_parity(dp, inst, v_term)
    print(f"{inst.name}: accepted near-tie policy mismatches = {n}")


@pytest.mark.parametrize("case", [dict(seed=21, T=3, K=2, S=32767, wu=7000, wd=7000),
                                  dict(seed=22, T=2, K=2, S=32767, wu=9000, wd=9000),
                                  dict(seed=23, T=2, K=1024, S=64, wu=8, wd=8)],
                         ids=["S_max_window_7000", "S_max_window_9000", "K_max"])
def test_maximum_sizes_match_oracle(dp, case):
    # S = DP_MAX_S with the widest windows the preferred tile and the one-wave fallback tile
    # hold in LDS, and K = DP_MAX_K
    kw = dict(case)
    seed, T, K, S, wu, wd = (kw.pop(k) for k in ("seed", "T", "K", "S", "wu", "wd"))
    inst = wl.random_small(seed, T, K, S, wu, wd, delta=0.001)
    n, V, pol, ref = full_parity(dp, inst)
    print(f"{inst.name}: accepted near-tie policy mismatches = {n}")


def test_hourly_day_small_matches_oracle(dp):
    inst = wl.day_hourly_small()
    n, V, pol, ref = full_parity(dp, inst)
    assert n <= 0.001 * pol.size


def test_five_minute_day_full_size_matches_oracle(dp):
    inst = wl.day_5min()
    n, V, pol, ref = full_parity(dp, inst)
    print(f"{inst.name}: accepted near-tie mismatches {n} of {pol.size}")
    # every mismatch already passed the near-tie rule; a systematic error would show as
    # far more of them
    assert n <= 0.01 * pol.size


def test_year_shapes_one_week_matches_oracle(dp):
    inst = wl.year_hourly(T=168)
    n, V, pol, ref = full_parity(dp, inst)
    print(f"{inst.name}: accepted near-tie mismatches {n} of {pol.size}")
    assert n <= 0.01 * pol.size


@pytest.mark.timeout(1200)
def test_year_full_horizon_matches_oracle_recursion(dp):
    """T = 8760, K = 50, S = 2001, +-500, start cost: every stage of the GPU solve against
    the oracle's own FP64 recursion run from V_{T+1} = 0 (no GPU value enters the oracle),
    so rounding accumulated over the whole horizon is measured.  Values per stage within
    the normwise tolerance; policies equal except at accepted near-ties, whose count and
    largest regret are reported and bounded."""
    from parity import STATS, _mismatch
    inst = wl.year_hourly()
    st, T, K, S = inst.storage, inst.T, inst.K, inst.storage.S
    out = gpu_solve(dp, inst, store_all=True)
    Vd, pold = out["V"], out["policy"]
    v_or = np.zeros((K, S))
    worst, n_mis, chunk = 0.0, 0, 240
    regret0 = STATS["max_regret"]
    STATS["max_regret"] = 0.0
    for hi in range(T, 0, -chunk):            # copy stages [lo, hi] (1-based) per chunk
        lo = max(1, hi - chunk + 1)
        v_blk = Vd[lo - 1:hi].cpu().numpy()
        p_blk = pold[lo - 1:hi].cpu().numpy()
        for t in range(hi, lo - 1, -1):
            v_new, p_or, W = oracle.stage(st, inst.lam[t - 1], inst.P[t - 1], v_or, want_w=True)
            err = value_error(v_blk[t - lo], v_new)
            worst = max(worst, err)
            assert err <= RTOL, f"year stage {t}: normwise value error {err:.3e}"
            n_mis += _mismatch(st, inst.lam[t - 1], inst.P[t - 1], v_or, v_new, p_blk[t - lo],
                               p_or, f"year stage {t}", W=W)
            v_or = v_new
        if hi % 2160 == 0 or lo == 1:
            print(f"year: stages {lo}..{T} checked, worst normwise error {worst:.2e}, "
                  f"accepted near-ties {n_mis}", flush=True)
    regret = STATS["max_regret"]
    STATS["max_regret"] = max(regret0, regret)
    print(f"year full horizon: worst normwise value error {worst:.2e}; accepted near-tie "
          f"mismatches {n_mis} of {T * K * S} ({n_mis / (T * K * S):.2e}); largest regret "
          f"{regret:.2e} of the stage scale")
    assert n_mis <= 0.01 * T * K * S
    assert regret <= RTOL
    del out, Vd, pold
    torch.cuda.empty_cache()


def test_year_full_size_sampled_stages(dp):
    """T = 8760: each sampled stage t is recomputed by the oracle from the GPU's V_{t+1}."""
    inst = wl.year_hourly()
    out = gpu_solve(dp, inst, store_all=True)
    Vd, pold = out["V"], out["policy"]
    T = inst.T
    for t in (T, T - 1, 6000, 4380, 1234, 2, 1):
        v_next = Vd[t].cpu().numpy().astype(np.float64)
        v_gpu = Vd[t - 1].cpu().numpy()
        p_gpu = pold[t - 1].cpu().numpy()
        check_stage(inst.storage, inst.lam[t - 1], inst.P[t - 1], v_next, v_gpu, p_gpu,
                    label=f"year stage {t}")
    assert np.all(np.isfinite(Vd[0].cpu().numpy()))
    del out, Vd, pold
    torch.cuda.empty_cache()


def test_v1_only_equals_all_stage_slice_bitwise(dp):
    inst = wl.random_small(21, 9, 12, 300, 30, 20, c_start=1.0)
    a = gpu_solve(dp, inst, store_all=True)
    b = gpu_solve(dp, inst, store_all=False, policy=False)
    assert torch.equal(a["V"][0], b["V"])


def test_repeat_runs_are_bitwise_identical(dp):
    inst = wl.day_hourly_small()
    a = gpu_solve(dp, inst, store_all=True)
    b = gpu_solve(dp, inst, store_all=True)
    assert torch.equal(a["V"], b["V"]) and torch.equal(a["policy"], b["policy"])


@pytest.mark.parametrize("shape", [(512, 8), (256, 8), (128, 8), (1024, 8), (960, 8), (448, 8),
                                   (1024, 4), (512, 4), (448, 4), (256, 4), (128, 4), (64, 4),
                                   (512, 2), (448, 2), (256, 2), (192, 2), (128, 2), (64, 2),
                                   (1024, 1), (512, 1), (448, 1), (256, 1), (192, 1), (128, 1),
                                   (64, 1)])
def test_tile_shapes_give_bitwise_identical_results(dp, shape):
    # the second instance has windows of 153 and 174 moves on 1966 levels: every tile then
    # holds windows wholly outside [0, S) at the edges, whose scans carry no position; the
    # third one's 51 moves take the direct maximum
    for inst in (wl.random_small(31, 6, 21, 1100, 260, 180, c_start=3.0, lam_lo=-60.0),
                 wl.random_small(32, 4, 10, 1966, 153, 174, c_start=1.0),
                 wl.random_small(33, 5, 7, 700, 30, 20, c_start=2.0)):
        dp.set_sweep_shape()
        ref = gpu_solve(dp, inst, store_all=True)
        try:
            dp.set_sweep_shape(*shape)
            got = gpu_solve(dp, inst, store_all=True)
        finally:
            dp.set_sweep_shape()
        assert torch.equal(ref["V"], got["V"]) and torch.equal(ref["policy"], got["policy"])


def test_checkpoint_buffer_does_not_change_results(dp):
    inst = wl.random_small(41, 40, 6, 200, 20, 20)
    a = gpu_solve(dp, inst, store_all=True)
    b = gpu_solve(dp, inst, store_all=True, ckpt_every=7)
    assert torch.equal(a["V"], b["V"]) and torch.equal(a["policy"], b["policy"])


def test_validation_rejects_non_stochastic_rows(dp):
    inst = wl.random_small(51, 3, 4, 10, 2, 2)
    P = inst.P.copy()
    P[1, 2, 0] += np.float32(0.01)
    with pytest.raises(dp.DPError) as e:
        dp.solve(dev(inst.lam), dev(P), inst.storage, validate=True)
    assert e.value.code == -2
    dp.solve(dev(inst.lam), dev(inst.P), inst.storage, validate=True)
    torch.cuda.synchronize()


def test_binding_checks_shapes_before_queueing(dp):
    inst = wl.random_small(61, 4, 3, 20, 2, 3)
    lam, P = dev(inst.lam), dev(inst.P)
    out = gpu_solve(dp, inst, store_all=True)
    seed = torch.zeros(3, 20, device="cuda")
    with pytest.raises(ValueError):
        dp.adjoint(lam, P, inst.storage, seed, V_all=out["V"][:-1], policy=out["policy"])
    with pytest.raises(TypeError):
        dp.adjoint(lam, P, inst.storage, seed, V_all=out["V"], policy=out["policy"].int())
    with pytest.raises(ValueError):
        dp.solve(lam, P[:, :2, :], inst.storage)
    with pytest.raises(ValueError):
        dp.solve(lam, P, inst.storage, v_term=torch.zeros(3, 19, device="cuda"))
    plan = dp.BatchPlan([(inst.T, inst.K, inst.storage)])
    with pytest.raises(ValueError):
        plan.solve([lam], [P], [torch.empty(3, 21, device="cuda")])
    with pytest.raises(ValueError):
        plan.solve([lam, lam], [P], [torch.empty(3, 20, device="cuda")])
    plan.close()


@pytest.mark.parametrize("which", ["T2000_K10", "year_week"])
def test_rows_off_the_simplex_match_oracle(dp, which):
    """Rows of P_t that sum to 1 only within ~2e-6 (unquantised, as estimated chains are):
    the offset carried between stages is multiplied by each row sum, so a solver that
    assumed unit sums would drift by about (row sum - 1) x (accumulated value) per stage."""
    base = (wl.random_small(71, 2000, 10, 101, 25, 25, c_start=0.5) if which == "T2000_K10"
            else wl.year_hourly(T=168))
    inst = dataclasses.replace(base, name=base.name + "_offsimplex",
                               P=wl.unnormalised_rows(base.P, 2e-6, seed=71))
    rs = inst.P.astype(np.float64).sum(-1)
    assert np.abs(rs - 1.0).max() > 1e-6
    n, V, pol, ref = full_parity(dp, inst)
    print(f"{inst.name}: accepted near-tie mismatches {n} of {pol.size}")
    assert n <= 0.01 * pol.size


def test_side_stream_solve_and_batch_equal_current_stream(dp):
    inst = wl.random_small(81, 20, 16, 400, 40, 40, c_start=1.0)
    ref = gpu_solve(dp, inst, store_all=True)
    side = torch.cuda.Stream()
    lam, P = dev(inst.lam), dev(inst.P)          # copies queued on the current stream
    out = dp.solve(lam, P, inst.storage, store_all=True, stream=side)
    plan = dp.BatchPlan([(inst.T, inst.K, inst.storage)], stream=side)
    V1 = torch.empty(inst.K, inst.storage.S, device="cuda")
    pol = torch.empty(inst.T, inst.K, inst.storage.S, dtype=torch.int16, device="cuda")
    plan.solve([lam], [P], [V1], [pol], stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert torch.equal(out["V"], ref["V"]) and torch.equal(out["policy"], ref["policy"])
    assert torch.equal(V1, ref["V"][0]) and torch.equal(pol, ref["policy"])
    plan.close()
