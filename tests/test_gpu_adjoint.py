"""GPU parity of the adjoint (dp_adjoint through the C ABI, and DPFunction autograd).

Reference: the FP64 oracle adjoint evaluated under the GPU's policies (the gradient of
the value of a fixed policy set), and central finite differences of the FP64 oracle at
points where the perturbation changes no policy.
"""
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


def test_adjoint_against_finite_differences(dp):
    """K=10, S=101, +-25, T=288 sub-instance; h = 2^-10 $/MWh on prices (exact in FP32).

    Two FP64 references: (a) central differences of the value of the GPU's policy set
    (J is linear in lam for fixed policies, so the difference quotient is exact), at
    every sampled point; (b) central differences of the optimal value, at points where
    neither perturbation changes the optimal policy and the GPU policy equals it.
    """
    inst = wl.fd_sub_5min()
    st = inst.storage
    om = wl.default_seed(inst.K, st.S)
    out, g = gpu_forward_backward(dp, inst, om)
    gl = g["grad_lam"].cpu().numpy()
    pol_gpu = out["policy"].cpu().numpy()
    base = oracle.solve(st, inst.lam, inst.P)
    same_policy = np.array_equal(pol_gpu, base["policy"])
    rng = np.random.default_rng(3)
    h = 2.0 ** -10
    tol = 1e-4 * max(1.0, float(np.max(np.abs(gl))))
    n_opt = 0
    for _ in range(24):
        t, k = int(rng.integers(0, inst.T)), int(rng.integers(0, inst.K))
        jp, jo = [], []
        stable = True
        for sgn in (1, -1):
            lam2 = inst.lam.copy()
            lam2[t, k] = np.float32(float(lam2[t, k]) + sgn * h)
            jp.append(float((om * oracle.policy_value(st, lam2, inst.P, pol_gpu)).sum()))
            o = oracle.solve(st, lam2, inst.P, keep_all=False)
            stable &= np.array_equal(o["policy"], base["policy"])
            jo.append(float((om * o["V1"]).sum()))
        fd_pol = (jp[0] - jp[1]) / (2 * h)
        assert abs(fd_pol - gl[t, k]) <= tol, (t, k, fd_pol, gl[t, k])
        if stable and same_policy:
            fd_opt = (jo[0] - jo[1]) / (2 * h)
            assert abs(fd_opt - gl[t, k]) <= tol, (t, k, fd_opt, gl[t, k])
            n_opt += 1
    print(f"FD points vs optimal value: {n_opt}; GPU policy equals oracle policy: {same_policy}")


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
