"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics.

Each test states what it pins.  None of them re-types the oracle's recursion: the
brute force enumerates plans, the LP is a different model, Algorithm 1 is the paper's
tensor formulation, the closed forms are derived by hand, the invariances follow from
the structure of the Bellman operator.
"""
import dataclasses
import math
import os

import numpy as np
import pytest

import oracle
from oracle import alg1, brute, hull, lp
import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(seed, T, K, S, wu, wd, **kw):
    return wl.random_small(seed, T, K, S, wu, wd, **kw)


# ---------------------------------------------------------------- P7: grid counts (paper tables)
def test_action_and_state_counts_match_paper_tables():
    eta = math.sqrt(0.85)
    seen = 0
    for line in open(os.path.join(GOLD, "grid_counts.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        kind, delta, dur, expected = line.split()
        delta, expected = float(delta), int(expected)
        if kind == "P":
            p, n_c, n_d = alg1.power_grid(1.0, delta, eta)
            assert p.shape[0] == expected == n_c + n_d + 1
            assert p[0] == -1.0 and p[-1] == 1.0 and 0.0 in p
        else:
            assert alg1.soc_grid(float(dur), delta).shape[0] == expected
        seen += 1
    assert seen == 10


# ---------------------------------------------------------------- P1: brute force on tiny trees
@pytest.mark.parametrize("case", [
    dict(seed=11, T=2, K=2, S=3, wu=2, wd=2),
    dict(seed=12, T=3, K=2, S=3, wu=1, wd=2),
    dict(seed=13, T=3, K=1, S=4, wu=3, wd=3),
    dict(seed=14, T=2, K=2, S=4, wu=2, wd=1, c_start=3.0),
    dict(seed=15, T=3, K=2, S=3, wu=2, wd=2, lam_lo=-120.0, lam_hi=30.0),
    dict(seed=16, T=2, K=3, S=3, wu=1, wd=1, eta=0.7, c_deg=4.0),
])
def test_backward_induction_equals_best_plan(case):
    kw = dict(case)
    seed, T, K, S, wu, wd = (kw.pop(k) for k in ("seed", "T", "K", "S", "wu", "wd"))
    inst = _rand(seed, T, K, S, wu, wd, **kw)
    rng = np.random.default_rng(seed)
    v_term = rng.uniform(-5, 5, size=(K, S)) if seed % 2 else None
    out = oracle.solve(inst.storage, inst.lam, inst.P, v_term)
    for k0 in range(K):
        for s0 in range(S):
            best, nplans = brute.best_plan_value(inst.storage, inst.lam, inst.P, s0, k0, v_term)
            assert nplans > 1
            assert abs(out["V1"][k0, s0] - best) <= 1e-12 * max(1.0, abs(best))


def test_backward_induction_equals_best_markov_policy():
    inst = _rand(21, 2, 2, 3, 1, 1, c_start=1.0)
    out = oracle.solve(inst.storage, inst.lam, inst.P)
    for k0 in range(2):
        for s0 in range(3):
            best = brute.best_markov_policy_value(inst.storage, inst.lam, inst.P, s0, k0)
            assert abs(out["V1"][k0, s0] - best) <= 1e-12 * max(1.0, abs(best))


def test_policy_attains_value_and_is_feasible():
    inst = _rand(22, 6, 3, 9, 3, 2, c_start=2.0)
    out = oracle.solve(inst.storage, inst.lam, inst.P)
    pol = out["policy"].astype(np.int64)
    s = np.arange(9)[None, None, :]
    assert np.all(pol >= np.maximum(0, s - 2)) and np.all(pol <= np.minimum(8, s + 3))
    v_pol = oracle.policy_value(inst.storage, inst.lam, inst.P, out["policy"])
    np.testing.assert_allclose(v_pol, out["V1"], rtol=0, atol=1e-10)


# ---------------------------------------------------------------- P2: LP bound / equality (K = 1)
def _det(seed, T, S, wu, wd, eta, c_deg, c_start, lo=-30.0, hi=90.0, delta=0.5):
    rng = np.random.default_rng(seed)
    lam = wl.f32(rng.uniform(lo, hi, size=(T, 1)))
    P = np.ones((T, 1, 1), np.float32)
    st = wl.Storage(S=S, w_up=wu, w_down=wd, delta=delta, eta_c=eta, eta_d=eta,
                    c_deg=c_deg, c_start=c_start).as_f32()
    return st, lam, P


@pytest.mark.parametrize("seed", range(5))
def test_dp_never_exceeds_lp(seed):
    st, lam, P = _det(100 + seed, 30, 9, 3, 2, 0.9, 1.5, 2.0 * (seed % 2), lo=-60.0)
    dp = oracle.solve(st, lam, P)["V1"][0, 0]
    lpv, _, _ = lp.arbitrage_lp(st, lam, s0=0)
    assert dp <= lpv + 1e-7 * max(1.0, abs(lpv))


@pytest.mark.parametrize("seed", range(5))
def test_dp_equals_lp_when_lossless_and_unimodular(seed):
    st, lam, P = _det(200 + seed, 40, 11, 3, 4, 1.0, 0.5 * seed, 0.0, lo=-40.0)
    dp = oracle.solve(st, lam, P)["V1"]
    for s0 in (0, 5, 10):
        lpv, _, _ = lp.arbitrage_lp(st, lam, s0=s0)
        assert abs(dp[0, s0] - lpv) <= 1e-7 * max(1.0, abs(lpv))


def test_gap_to_lp_shrinks_with_finer_grid():
    # Sec. V-A: the discretised DP is a restriction and its gap to the LP shrinks
    # roughly linearly with delta.  1 MW / 1 MWh battery, eta = sqrt(0.85); the LP has the
    # power limit (SoC moves eta and 1/eta per stage), the DP the largest whole-step window
    # inside it, so the DP cannot use the fractional end of the power range.
    rng = np.random.default_rng(7)
    T = 48
    lam = wl.f32(40 + 25 * np.sin(np.arange(T) * 2 * np.pi / 24) + rng.normal(0, 5, T)).reshape(T, 1)
    P = np.ones((T, 1, 1), np.float32)
    eta = math.sqrt(0.85)
    gaps = []
    for n in (5, 10, 20, 50, 100):
        delta = 1.0 / n
        st = wl.Storage(S=n + 1, w_up=int(math.floor(eta / delta + 1e-9)),
                        w_down=int(math.floor(1.0 / (eta * delta) + 1e-9)), delta=delta,
                        eta_c=eta, eta_d=eta, c_deg=1.0).as_f32()
        dp = oracle.solve(st, lam, P, keep_all=False, want_policy=False)["V1"][0, 0]
        st_lp = dataclasses.replace(st, w_up=eta / st.delta, w_down=1.0 / (eta * st.delta))
        lpv, _, _ = lp.arbitrage_lp(st_lp, lam)
        assert dp <= lpv + 1e-7
        gaps.append((lpv - dp) / lpv)
    assert gaps[0] > 1e-3
    assert gaps[-1] < gaps[0] / 5 and gaps[-1] < 0.01


# ---------------------------------------------------------------- P3: monotone / concave in SoC
def test_monotone_and_concave_when_prices_above_minus_cdeg():
    inst = _rand(31, 12, 4, 30, 5, 6, c_deg=3.0, lam_lo=-2.9, lam_hi=90.0)
    V = oracle.solve(inst.storage, inst.lam, inst.P)["V"]
    d1 = np.diff(V, axis=-1)
    assert np.all(d1 >= -1e-9)
    assert np.all(np.diff(d1, axis=-1) <= 1e-9)


def test_monotone_with_start_cost():
    inst = _rand(32, 10, 3, 25, 4, 4, c_deg=1.0, c_start=7.0, lam_lo=0.0, lam_hi=80.0)
    V = oracle.solve(inst.storage, inst.lam, inst.P)["V"]
    assert np.all(np.diff(V, axis=-1) >= -1e-9)


def test_value_can_decrease_in_soc_at_negative_prices():
    # Sec. II-C: with sufficiently negative prices headroom is worth more than energy.
    st = wl.Storage(S=5, w_up=4, w_down=4, delta=1.0, eta_c=0.9, eta_d=0.9).as_f32()
    lam = np.array([[-50.0], [-50.0]], np.float32)
    P = np.ones((2, 1, 1), np.float32)
    V = oracle.solve(st, lam, P)["V1"][0]
    assert V[0] > V[-1]


# ---------------------------------------------------------------- P4: stochastic rows
def test_generated_rows_are_exactly_stochastic():
    for inst in (wl.day_hourly_small(), wl.day_5min(T=12), wl.year_hourly(T=30)):
        P = inst.P.astype(np.float64)
        assert np.all(P >= 0)
        assert np.all(P.sum(-1) == 1.0)
        assert np.all(np.rint(P * 2.0 ** 24) == P * 2.0 ** 24)


# ---------------------------------------------------------------- P5: Algorithm 1 special case
@pytest.mark.parametrize("eta", [1.0, 0.9])
def test_markov_dp_reduces_to_algorithm1(eta):
    rng = np.random.default_rng(41)
    T, R, S, W = 8, 5, 21, 4
    delta = 0.25
    lam = wl.f32(rng.uniform(-30, 90, size=(T, R)))
    pi = wl.quantize_rows(rng.dirichlet(np.ones(R), size=T)).astype(np.float64)
    # P_t rows all equal pi_{t+1} (stagewise independence); P_T multiplies V_{T+1} = 0.
    P = np.empty((T, R, R), np.float32)
    for t in range(T):
        P[t] = pi[t + 1] if t + 1 < T else pi[t]
    st = wl.Storage(S=S, w_up=W, w_down=W, delta=delta, eta_c=eta, eta_d=eta).as_f32()
    Vm = oracle.solve(st, lam, P)["V"]
    # Alg. 1 with the integer-step action grid (no interpolated endpoints)
    p_hat = np.array([-(k * st.delta / st.eta_c) for k in range(W, 0, -1)] + [0.0] +
                     [k * st.delta * st.eta_d for k in range(1, W + 1)])
    s_hat = np.arange(S) * st.delta
    Va = alg1.algorithm1(s_hat, p_hat, lam, pi, st.eta_c)
    for t in range(1, T + 1):
        expect = (pi[t - 1][:, None] * Vm[t - 1]).sum(0)        # sum_k pi_t[k] V^M_t[k, :]
        np.testing.assert_allclose(Va[t - 1], expect, rtol=1e-12, atol=1e-9)


def test_algorithm1_interpolated_endpoints_bounded_by_lp():
    # Deterministic R = 1, paper power grid with fractional endpoints: still a restriction.
    rng = np.random.default_rng(43)
    T = 24
    lam = wl.f32(rng.uniform(-10, 80, size=(T, 1)))
    eta = math.sqrt(0.85)
    delta = 0.1
    s_hat = alg1.soc_grid(1.0, delta)
    p_hat, _, _ = alg1.power_grid(1.0, delta, eta)
    V = alg1.algorithm1(s_hat, p_hat, lam, np.ones((T, 1)), eta)
    st = wl.Storage(S=s_hat.shape[0], w_up=100, w_down=100, delta=delta, eta_c=eta,
                    eta_d=eta).as_f32()
    # LP with the power limit p_bar = 1 expressed as SoC-move limits eta and 1/eta.
    st_lp = dataclasses.replace(st, w_up=eta / delta, w_down=1.0 / (eta * delta))
    lpv, _, _ = lp.arbitrage_lp(st_lp, lam)
    assert V[0, 0] <= lpv + 1e-7
    assert V[0, 0] >= 0.9 * lpv


# ---------------------------------------------------------------- P6: closed forms
def test_zero_window_gives_zero_value():
    inst = _rand(51, 5, 3, 7, 0, 0, c_start=1.0)
    out = oracle.solve(inst.storage, inst.lam, inst.P)
    assert np.all(out["V"] == 0.0)
    assert np.all(out["policy"] == np.arange(7)[None, None, :])


def test_single_stage_is_myopic_best_move():
    st = wl.Storage(S=6, w_up=2, w_down=3, delta=0.5, eta_c=0.8, eta_d=0.9, c_deg=1.0,
                    c_start=0.5).as_f32()
    lam = np.array([[30.0, -70.0]], np.float32)
    P = wl.quantize_rows(np.full((1, 2, 2), 0.5))
    V = oracle.solve(st, lam, P)["V1"]
    d, e = st.delta, st.eta_c
    # hand-derived: at +30 $/MWh sell as much as possible (discharge), at -70 $/MWh buy.
    for s in range(6):
        m = min(3, s)
        best_sell = 0.0 if m == 0 else m * d * st.eta_d * (30.0 - 1.0) - 0.5
        assert abs(V[0, s] - max(0.0, best_sell)) < 1e-9
        c = min(2, 5 - s)
        best_buy = 0.0 if c == 0 else c * d / e * (70.0 - 1.0) - 0.5
        assert abs(V[1, s] - max(0.0, best_buy)) < 1e-9


@pytest.mark.parametrize("eta_c,eta_d", [(0.9, 0.8), (0.75, 0.95), (1.0, 1.0)])
def test_two_stage_buy_low_sell_high(eta_c, eta_d):
    # K=1, T=2, from s0=0: charge m steps at lambda_1, discharge them at lambda_2.
    st = wl.Storage(S=8, w_up=3, w_down=5, delta=0.25, eta_c=eta_c, eta_d=eta_d,
                    c_deg=2.0).as_f32()
    lam = np.array([[20.0], [95.0]], np.float32)
    P = np.ones((2, 1, 1), np.float32)
    V = oracle.solve(st, lam, P)["V1"][0, 0]
    m = min(3, 5, 7)
    l1, l2, cd = 20.0, 95.0, st.c_deg
    expect = max(0.0, m * st.delta * (l2 * st.eta_d - l1 / st.eta_c - cd * (st.eta_d + 1 / st.eta_c)))
    assert abs(V - expect) < 1e-10


# ---------------------------------------------------------------- P8: invariances
def test_terminal_shift_shifts_values():
    inst = _rand(61, 6, 4, 12, 3, 3, c_start=2.0)
    rng = np.random.default_rng(0)
    vt = rng.uniform(-10, 10, size=(4, 12))
    a = oracle.solve(inst.storage, inst.lam, inst.P, vt)
    b = oracle.solve(inst.storage, inst.lam, inst.P, vt + 1234.5)
    np.testing.assert_allclose(b["V"], a["V"] + 1234.5, rtol=0, atol=1e-9)
    assert np.array_equal(a["policy"], b["policy"])


def test_price_scaling_by_two_is_exact():
    inst = _rand(62, 7, 3, 10, 2, 4, c_deg=0.0)
    a = oracle.solve(inst.storage, inst.lam, inst.P)
    b = oracle.solve(inst.storage, inst.lam * 2, inst.P)
    assert np.array_equal(b["V"], 2.0 * a["V"])
    assert np.array_equal(a["policy"], b["policy"])


def test_state_relabelling_permutes_values():
    inst = _rand(63, 5, 5, 8, 2, 2, c_start=1.0)
    perm = np.array([3, 0, 4, 1, 2])
    lam2 = inst.lam[:, perm]
    P2 = inst.P[:, perm][:, :, perm]
    a = oracle.solve(inst.storage, inst.lam, inst.P)
    b = oracle.solve(inst.storage, lam2, P2)
    np.testing.assert_allclose(b["V"], a["V"][:, perm], rtol=1e-13, atol=1e-9)


def test_split_solve_equals_whole_solve_bitwise():
    inst = _rand(64, 10, 3, 9, 3, 3, c_start=1.0)
    whole = oracle.solve(inst.storage, inst.lam, inst.P)
    t0 = 6                                               # solve stages 7..10, then 1..6
    tail = oracle.solve(inst.storage, inst.lam[t0:], inst.P[t0:])
    head = oracle.solve(inst.storage, inst.lam[:t0], inst.P[:t0], tail["V1"])
    assert np.array_equal(head["V1"], whole["V1"])
    assert np.array_equal(np.concatenate([head["policy"], tail["policy"]]), whole["policy"])


# ---------------------------------------------------------------- P9 / P10: adjoint
def _fd_ok(st, lam, P, seed, h, which, idx, threads=1):
    """Central FD of J at +-h on one FP32 input entry; None if the policies change.

    h is a power of two small enough that lam +- h and P +- h stay exactly
    representable in FP32, so the perturbed problems are exact inputs.
    """
    base = oracle.solve(st, lam, P, threads=threads)
    vals = []
    for sgn in (+1, -1):
        l2, P2 = lam.copy(), P.copy()
        if which == "lam":
            l2[idx] = np.float32(float(l2[idx]) + sgn * h)
            assert float(l2[idx]) == float(lam[idx]) + sgn * h
        else:
            P2[idx] = np.float32(float(P2[idx]) + sgn * h)
            assert float(P2[idx]) == float(P[idx]) + sgn * h
        o = oracle.solve(st, l2, P2, threads=threads)
        if not np.array_equal(o["policy"], base["policy"]):
            return None
        vals.append(float((seed * o["V1"]).sum()))
    return (vals[0] - vals[1]) / (2 * h)


def test_envelope_gradient_is_path_energy():
    # K = 1: dJ/dlambda_t = g(move taken at t) along the optimal path from s0 = 0.
    st, lam, P = _det(71, 20, 9, 3, 2, 0.9, 1.0, 0.0)
    out = oracle.solve(st, lam, P)
    seed = np.zeros((1, st.S)); seed[0, 0] = 1.0
    adj = oracle.adjoint(st, lam, P, out["V"], out["policy"], seed)
    s = 0
    for t in range(20):
        j = int(out["policy"][t, 0, s]); d = j - s
        g = -d * st.delta / st.eta_c if d > 0 else (-d * st.delta * st.eta_d if d < 0 else 0.0)
        assert abs(adj["grad_lam"][t, 0] - g) < 1e-12
        s = j


@pytest.mark.parametrize("seed_", [0, 1])
def test_adjoint_matches_central_differences(seed_):
    inst = _rand(80 + seed_, 6, 3, 9, 3, 2, c_start=1.0 * seed_)
    st = inst.storage
    out = oracle.solve(st, inst.lam, inst.P)
    om = np.random.default_rng(seed_).uniform(0, 1, size=(3, 9))
    adj = oracle.adjoint(st, inst.lam, inst.P, out["V"], out["policy"], om)
    checked = 0
    for t in range(6):
        for k in range(3):
            fd = _fd_ok(st, inst.lam, inst.P, om, 2.0 ** -10, "lam", (t, k))
            if fd is not None:
                assert abs(fd - adj["grad_lam"][t, k]) <= 1e-9 * max(1.0, abs(fd))
                checked += 1
            for kp in range(3):
                fd = _fd_ok(st, inst.lam, inst.P, om, 2.0 ** -20, "P", (t, k, kp))
                if fd is not None:
                    assert abs(fd - adj["grad_P"][t, k, kp]) <= 1e-7 * max(1.0, abs(fd))
                    checked += 1
    assert checked > 30


def test_adjoint_conserves_mass_and_gives_terminal_gradient():
    inst = _rand(90, 8, 4, 11, 3, 3, c_start=2.0)
    st = inst.storage
    rng = np.random.default_rng(1)
    vt = rng.uniform(-3, 3, size=(4, 11))
    out = oracle.solve(st, inst.lam, inst.P, vt)
    om = rng.uniform(0, 1, size=(4, 11))
    adj = oracle.adjoint(st, inst.lam, inst.P, out["V"], out["policy"], om)
    assert abs(adj["grad_vterm"].sum() - om.sum()) < 1e-12 * om.sum() * 10
    # J is linear in v_term for fixed policies: J(v + e) - J(v) = <grad, e>
    e = rng.uniform(-1, 1, size=(4, 11))
    j0 = (om * oracle.policy_value(st, inst.lam, inst.P, out["policy"], vt)).sum()
    j1 = (om * oracle.policy_value(st, inst.lam, inst.P, out["policy"], vt + e)).sum()
    assert abs((j1 - j0) - (adj["grad_vterm"] * e).sum()) < 1e-9


# ---------------------------------------------------------------- hull oracle vs SciPy
def test_envelope_definition_matches_scipy_hull():
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(5)
    xs = np.sort(rng.uniform(-1, 1, 15))
    ys = rng.normal(0, 1, 15) - 2 * xs ** 2
    pts = np.column_stack([xs, ys])
    bottom = np.array([[xs[0], ys.min() - 10], [xs[-1], ys.min() - 10]])
    h = ConvexHull(np.vstack([pts, bottom]))
    vert = sorted(i for i in h.vertices if i < 15)
    for i in range(15):
        env = hull.envelope_at(xs, ys, xs[i])
        on_hull = i in vert
        assert (abs(env - ys[i]) < 1e-12) == on_hull


# ---------------------------------------------------------------- tie-break reading
def test_ties_resolve_to_smallest_next_state():
    # With zero prices and costs every feasible move is worth 0: the documented tie-break
    # (first maximum in ascending j) must pick the lowest reachable SoC.
    st = wl.Storage(S=12, w_up=3, w_down=4, delta=0.5, eta_c=0.9, eta_d=0.9).as_f32()
    lam = np.zeros((4, 2), np.float32)
    P = wl.quantize_rows(np.full((4, 2, 2), 0.5))
    out = oracle.solve(st, lam, P)
    assert np.all(out["V"] == 0.0)
    s = np.arange(12)
    assert np.all(out["policy"] == np.maximum(0, s - 4)[None, None, :])


# ---------------------------------------------------------------- tie-break in Algorithm 1's oracle
def test_algorithm1_policy_index_breaks_ties_to_smallest_next_state():
    # Hand-built Q tensors (S x P x R) with exact ties: the index returned must be the
    # largest maximising action on the ascending power grid; -inf (infeasible) is never
    # chosen and a unique maximum is returned as it is.
    q = np.array([[[1.0], [3.0], [3.0], [2.0]],           # tie between 1 and 2 -> 2
                  [[5.0], [-np.inf], [4.0], [-np.inf]],   # unique maximum at 0
                  [[0.0], [0.0], [0.0], [-np.inf]],       # tie 0, 1, 2; 3 infeasible -> 2
                  [[7.0], [7.0], [7.0], [7.0]]])          # all tied -> 3
    assert alg1.policy_index(q)[:, 0].tolist() == [2, 0, 2, 3]
    # Through Algorithm 1 itself: with zero prices and a zero continuation every feasible
    # action is worth 0, so the chosen action must be the feasible one with the smallest
    # next state, computed here from the transition F of Eq. (2) directly.
    eta, delta = 0.9, 0.1
    s_hat = alg1.soc_grid(1.0, delta)
    p_hat, _, _ = alg1.power_grid(0.35, delta, eta)
    pre = alg1.precompute(s_hat, p_hat, eta)
    _, Q_all = alg1.stage(pre, p_hat, np.zeros(2), np.array([0.5, 0.5]), np.zeros(s_hat.size))
    pol = alg1.policy_index(Q_all)
    for s in range(s_hat.size):
        nxt = np.array([s_hat[s] + (-p / eta if p >= 0 else -eta * p) for p in p_hat])
        ok = (nxt >= -1e-9) & (nxt <= s_hat[-1] + 1e-9)
        best = int(np.flatnonzero(ok)[np.argmin(nxt[ok])])
        assert pol[s].tolist() == [best, best], (s, pol[s], best)


# ---------------------------------------------------------------- candidate lookup used by the near-tie rule
def test_candidate_lookup_attains_the_stage_maximum():
    # q_at(k, s, j) must equal the stage value at the oracle's own argmax, never exceed it
    # at any feasible move, and be -inf exactly outside J(s).
    inst = _rand(5, 3, 4, 50, 6, 7, c_start=1.0, lam_lo=-60.0)
    st = inst.storage
    v = np.random.default_rng(0).normal(size=(4, 50))
    V, pol, W = oracle.stage(st, inst.lam[0], inst.P[0], v, want_w=True)
    k, s = np.meshgrid(np.arange(4), np.arange(50), indexing="ij")
    k, s = k.ravel(), s.ravel()
    np.testing.assert_allclose(oracle.q_at(st, inst.lam[0], W, k, s, pol[k, s]), V[k, s],
                               rtol=0, atol=1e-12)
    for j in range(50):
        q = oracle.q_at(st, inst.lam[0], W, k, s, np.full_like(k, j))
        feas = (j >= s - st.w_down) & (j <= s + st.w_up)
        assert np.all(np.isinf(q[~feas])) and np.all(np.isfinite(q[feas]))
        assert np.all(q[feas] <= V[k, s][feas] + 1e-12)
