"""GPU parity of the adjoint (dp_adjoint through the C ABI, and DPFunction autograd).

Reference: the FP64 oracle adjoint evaluated under the GPU's policies (the gradient of
the value of a fixed policy set), and central finite differences of the FP64 oracle at
points where the perturbation changes no policy.
"""
import dataclasses

import numpy as np
import pytest

import oracle
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def normwise(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-30)
    return float(np.max(np.abs(a.astype(np.float64) - b))) / scale


def gpu_forward_backward(dp, inst, seed, ckpt_every=0):
    lam, P = dev(inst.lam), dev(inst.P)
    if ckpt_every:
        out = dp.solve(lam, P, inst.storage, store_all=False, policy=False, ckpt_every=ckpt_every)
        g = dp.adjoint(lam, P, inst.storage, dev(seed), ckpt=out["ckpt"], ckpt_every=ckpt_every,
                       want_vterm=True)
    else:
        out = dp.solve(lam, P, inst.storage, store_all=True, policy=True)
        g = dp.adjoint(lam, P, inst.storage, dev(seed), V_all=out["V"], policy=out["policy"],
                       want_vterm=True)
    torch.cuda.synchronize()
    return out, g


def oracle_under_gpu_policy(inst, pol_gpu, seed):
    """FP64 adjoint for the GPU's policies: values of that policy set, then the adjoint."""
    st = inst.storage
    T, K = inst.lam.shape
    # values of the fixed policy at every stage (backward policy evaluation, stage by stage)
    V = np.zeros((T + 1, K, st.S))
    for t in range(T, 0, -1):
        V[t - 1] = oracle.policy_value(st, inst.lam[t - 1:t], inst.P[t - 1:t], pol_gpu[t - 1:t],
                                       V[t])
    return oracle.adjoint(st, inst.lam, inst.P, V, pol_gpu, seed.astype(np.float64))


CASES = [
    dict(seed=1, T=6, K=3, S=40, wu=5, wd=7, c_start=1.0),
    dict(seed=2, T=10, K=17, S=300, wu=30, wd=45),
    dict(seed=3, T=5, K=20, S=1001, wu=250, wd=250, lam_lo=-150.0),
    dict(seed=4, T=4, K=1, S=9, wu=2, wd=3),
    dict(seed=5, T=1, K=4, S=30, wu=3, wd=4, c_start=0.5),    # a single stage
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"s{c['seed']}_K{c['K']}_S{c['S']}")
def test_adjoint_matches_oracle_under_gpu_policy(dp, case):
    kw = dict(case)
    seed_, T, K, S, wu, wd = (kw.pop(k) for k in ("seed", "T", "K", "S", "wu", "wd"))
    inst = wl.random_small(seed_, T, K, S, wu, wd, **kw)
    om = np.random.default_rng(seed_).uniform(0, 1, size=(K, S)).astype(np.float32)
    out, g = gpu_forward_backward(dp, inst, om)
    ref = oracle_under_gpu_policy(inst, out["policy"].cpu().numpy(), om)
    assert normwise(g["grad_lam"].cpu().numpy(), ref["grad_lam"]) <= RTOL
    assert normwise(g["grad_P"].cpu().numpy(), ref["grad_P"]) <= RTOL
    assert normwise(g["grad_vterm"].cpu().numpy(), ref["grad_vterm"]) <= RTOL


def test_adjoint_with_rows_off_the_simplex_matches_oracle(dp):
    # rows summing to 1 only within 2e-6: the forward values carry the row sums exactly,
    # and the gradients are the raw partials of that forward map
    base = wl.random_small(6, 40, 12, 200, 20, 30, c_start=1.0)
    inst = dataclasses.replace(base, P=wl.unnormalised_rows(base.P, 2e-6, seed=6))
    om = np.random.default_rng(6).uniform(0, 1, size=(12, 200)).astype(np.float32)
    out, g = gpu_forward_backward(dp, inst, om)
    ref = oracle_under_gpu_policy(inst, out["policy"].cpu().numpy(), om)
    for key in ("grad_lam", "grad_P", "grad_vterm"):
        assert normwise(g[key].cpu().numpy(), ref[key]) <= RTOL, key


def test_adjoint_full_size_day(dp):
    inst = wl.day_5min_adjoint()
    om = wl.default_seed(inst.K, inst.storage.S)
    out, g = gpu_forward_backward(dp, inst, om)
    ref = oracle_under_gpu_policy(inst, out["policy"].cpu().numpy(), om)
    e1 = normwise(g["grad_lam"].cpu().numpy(), ref["grad_lam"])
    e2 = normwise(g["grad_P"].cpu().numpy(), ref["grad_P"])
    print(f"full-size adjoint: grad_lam err {e1:.2e}, grad_P err {e2:.2e}")
    assert e1 <= RTOL and e2 <= RTOL


def test_checkpointed_adjoint_is_bitwise_equal_to_full_storage(dp):
    inst = wl.random_small(11, 37, 9, 150, 20, 25, c_start=2.0)
    om = np.random.default_rng(0).uniform(0, 1, size=(9, 150)).astype(np.float32)
    _, g_full = gpu_forward_backward(dp, inst, om, 0)
    for every in (1, 5, 16, 37, 50):
        out, g_ck = gpu_forward_backward(dp, inst, om, every)
        for key in ("grad_lam", "grad_P", "grad_vterm"):
            assert torch.equal(g_full[key], g_ck[key]), (every, key)


def test_checkpointed_adjoint_full_day_is_bitwise_equal(dp):
    # 18 segments of 16 stages: the re-solves alternate between two segment buffers on a
    # second stream while the adjoint of the previous segment runs; repeated twice so a
    # later call reuses the library's stream and the segment buffers' contents
    inst = wl.day_5min_adjoint()
    om = wl.default_seed(inst.K, inst.storage.S)
    _, g_full = gpu_forward_backward(dp, inst, om, 0)
    for rep in range(2):
        _, g_ck = gpu_forward_backward(dp, inst, om, 16)
        for key in ("grad_lam", "grad_P", "grad_vterm"):
            assert torch.equal(g_full[key], g_ck[key]), (rep, key)


def test_adjoint_is_deterministic(dp):
    inst = wl.random_small(12, 12, 30, 700, 90, 60)
    om = np.random.default_rng(1).uniform(0, 1, size=(30, 700)).astype(np.float32)
    _, a = gpu_forward_backward(dp, inst, om)
    _, b = gpu_forward_backward(dp, inst, om)
    for key in ("grad_lam", "grad_P", "grad_vterm"):
        assert torch.equal(a[key], b[key])


def fd_checks(inst, om, gl, gP, pol_gpu, *, n_lam=24, n_P=8, min_opt=4, seed=3):
    """Central differences of FP64 oracle objectives against the GPU gradients.

    (a) The value of the GPU's policy set, J_pi(lam, P) = sum om * V1_pi: for fixed policies
        it is linear in each lam_t[k] and each P_t[k][k'], so the difference quotient is
        exact; checked at every sampled point, for prices and for single entries of P
        (raw partials: the perturbed row is not renormalised).
    (b) The optimal value J*(lam), at price points where it is differentiable along the
        perturbation and the GPU's gradient is the derivative of J*: the oracle's optimal
        policy stays optimal at lam +- h (J* = J_pi_or there, to rounding), and the GPU's
        policies give the same derivative at that point as the oracle's (the two policy
        sets agree wherever the occupation measure reaching (t, k) has mass).  Points
        near t = 1 are included, where that measure is concentrated on few states.
    Returns the number of points compared in (b)."""
    st = inst.storage
    base = oracle.solve(st, inst.lam, inst.P)
    pol_or = base["policy"]
    om64 = om.astype(np.float64)
    g_or = oracle.adjoint(st, inst.lam, inst.P, base["V"], pol_or, om64)["grad_lam"]
    g_gp = oracle_under_gpu_policy(inst, pol_gpu, om)["grad_lam"]
    J = lambda lam, P, pol: float((om64 * oracle.policy_value(st, lam, P, pol)).sum())
    rng = np.random.default_rng(seed)
    h = 2.0 ** -10
    tol = 1e-4 * max(1.0, float(np.max(np.abs(gl))))
    scale = max(abs(J(inst.lam, inst.P, pol_or)), 1.0)
    n_opt = 0
    for n in range(n_lam):
        t = int(rng.integers(0, 4)) if n % 3 == 0 else int(rng.integers(0, inst.T))
        k = int(rng.integers(0, inst.K))
        jp, jo, jor = [], [], []
        for sgn in (1, -1):
            lam2 = inst.lam.copy()
            lam2[t, k] = np.float32(float(lam2[t, k]) + sgn * h)
            jp.append(J(lam2, inst.P, pol_gpu))
            jor.append(J(lam2, inst.P, pol_or))
            jo.append(float((om64 * oracle.solve(st, lam2, inst.P, keep_all=False)["V1"]).sum()))
        fd_pol = (jp[0] - jp[1]) / (2 * h)
        assert abs(fd_pol - gl[t, k]) <= tol, ("lam", t, k, fd_pol, gl[t, k])
        stays_optimal = all(abs(a - b) <= 1e-12 * scale for a, b in zip(jo, jor))
        same_derivative = abs(g_or[t, k] - g_gp[t, k]) <= 1e-12 * max(1.0, abs(g_or[t, k]))
        if stays_optimal and same_derivative:
            fd_opt = (jo[0] - jo[1]) / (2 * h)
            assert abs(fd_opt - gl[t, k]) <= tol, ("opt", t, k, fd_opt, gl[t, k])
            n_opt += 1
    tolP = 1e-4 * max(1.0, float(np.max(np.abs(gP))))
    hP = 2.0 ** -12          # P +- hP is exact in FP32 for entries on the 2^-24 grid
    for _ in range(n_P):
        t, k, kp = (int(rng.integers(0, m)) for m in (inst.T, inst.K, inst.K))
        jp = []
        for sgn in (1, -1):
            P2 = inst.P.copy()
            P2[t, k, kp] = np.float32(float(P2[t, k, kp]) + sgn * hP)
            jp.append(J(inst.lam, P2, pol_gpu))
        fd = (jp[0] - jp[1]) / (2 * hP)
        assert abs(fd - gP[t, k, kp]) <= tolP, ("P", t, k, kp, fd, gP[t, k, kp])
    assert n_opt >= min_opt, f"only {n_opt} points where the optimal value is differentiable"
    return n_opt


def test_adjoint_against_finite_differences(dp):
    """K=10, S=101, +-25, T=288 sub-instance; h = 2^-10 $/MWh on prices, 2^-12 on P."""
    inst = wl.fd_sub_5min()
    om = wl.default_seed(inst.K, inst.storage.S)
    out, g = gpu_forward_backward(dp, inst, om)
    n_opt = fd_checks(inst, om, g["grad_lam"].cpu().numpy(), g["grad_P"].cpu().numpy(),
                      out["policy"].cpu().numpy())
    print(f"FD points compared with the optimal value's derivative: {n_opt}")


def test_autograd_function_matches_direct_adjoint(dp):
    inst = wl.random_small(13, 8, 6, 64, 8, 8, c_start=0.5)
    lam = dev(inst.lam).requires_grad_(True)
    P = dev(inst.P).requires_grad_(True)
    om = torch.rand(6, 64, device="cuda")
    for every in (0, 3):
        V1 = dp.DPFunction.apply(lam, P, inst.storage, every)
        gl, gP = torch.autograd.grad((V1 * om).sum(), (lam, P))
        out = dp.solve(lam.detach(), P.detach(), inst.storage, store_all=True)
        d = dp.adjoint(lam.detach(), P.detach(), inst.storage, om, V_all=out["V"],
                       policy=out["policy"])
        assert torch.equal(gl, d["grad_lam"]) and torch.equal(gP, d["grad_P"])
        assert torch.equal(V1.detach(), out["V"][0])


@pytest.mark.parametrize("S", [16385, 32767])
def test_adjoint_beyond_one_accumulator_chunk_matches_oracle(dp, S):
    # the push-forward holds 16384 next states in LDS at a time: a row of 16385 takes two
    # passes (the second of one state), the largest grid two passes of 16384 and 16383;
    # moves of +-300 cross the chunk boundary
    inst = wl.random_small(20 + S % 7, 3, 2, S, 300, 300, delta=0.001, c_start=0.5)
    om = np.random.default_rng(S).uniform(0, 1, size=(2, S)).astype(np.float32)
    out, g = gpu_forward_backward(dp, inst, om)
    ref = oracle_under_gpu_policy(inst, out["policy"].cpu().numpy(), om)
    for key in ("grad_lam", "grad_P", "grad_vterm"):
        assert normwise(g[key].cpu().numpy(), ref[key]) <= RTOL, key


def test_validation_rejects_infeasible_policies(dp):
    inst = wl.random_small(14, 5, 3, 50, 4, 6)
    lam, P = dev(inst.lam), dev(inst.P)
    out = dp.solve(lam, P, inst.storage, store_all=True)
    seed = torch.rand(3, 50, device="cuda")
    ok = dp.adjoint(lam, P, inst.storage, seed, V_all=out["V"], policy=out["policy"], validate=True)
    bad = out["policy"].clone()
    bad[2, 1, 10] = 10 + 5          # beyond w_up = 4
    with pytest.raises(dp.DPError) as e:
        dp.adjoint(lam, P, inst.storage, seed, V_all=out["V"], policy=bad, validate=True)
    assert e.value.code == -1 and "feasible" in str(e.value)
    bad[2, 1, 10] = -1              # outside [0, S): no mass moves, nothing is written there
    g = dp.adjoint(lam, P, inst.storage, seed, V_all=out["V"], policy=bad)
    torch.cuda.synchronize()
    assert torch.isfinite(g["grad_P"]).all() and torch.isfinite(ok["grad_P"]).all()


def test_side_stream_adjoint_equals_current_stream(dp):
    inst = wl.random_small(15, 12, 8, 300, 30, 30, c_start=1.0)
    om = np.random.default_rng(2).uniform(0, 1, size=(8, 300)).astype(np.float32)
    _, ref = gpu_forward_backward(dp, inst, om)
    side = torch.cuda.Stream()
    lam, P, seed = dev(inst.lam), dev(inst.P), dev(om)      # copies queued on the current stream
    out = dp.solve(lam, P, inst.storage, store_all=True, stream=side)
    g = dp.adjoint(lam, P, inst.storage, seed, V_all=out["V"], policy=out["policy"],
                   want_vterm=True, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for key in ("grad_lam", "grad_P", "grad_vterm"):
        assert torch.equal(g[key], ref[key]), key
