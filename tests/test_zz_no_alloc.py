"""dp_solve_noalloc (solver state in the library's own device array) against dp_solve (a
caller workspace), through the C ABI: bitwise equal values and policies on two calls in a
row, the second smaller, and the size and flag rejections."""
import numpy as np
import pytest

import workloads as wl

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


def both(dp, inst, store_all):
    lam, P = dev(inst.lam), dev(inst.P)
    K, S, T = inst.K, inst.storage.S, inst.T
    ref = dp.solve(lam, P, inst.storage, store_all=store_all, policy=True)
    V = torch.full((T + 1, K, S) if store_all else (K, S), float("nan"), device="cuda")
    pol = torch.full((T, K, S), -7, dtype=torch.int16, device="cuda")
    dp.solve_noalloc(lam, P, inst.storage, V, pol, store_all=store_all)
    torch.cuda.synchronize()
    assert torch.equal(ref["V"], V), f"{inst.name}: values differ"
    assert torch.equal(ref["policy"], pol), f"{inst.name}: policies differ"


def test_noalloc_equals_workspace_solve_on_two_calls_second_smaller(dp):
    day = wl.day_5min()
    big = wl.Instance(day.name + "_T24", 24, day.K, day.storage, day.lam[:24], day.P[:24])
    small = wl.random_small(77, 7, 10, 101, 25, 25, c_start=1.0)
    both(dp, big, store_all=True)         # 100 x 1001, all stages
    both(dp, small, store_all=False)      # then a smaller problem, V_1 only
    both(dp, small, store_all=True)


def test_noalloc_year_shapes_equal_workspace_solve(dp):
    year = wl.year_hourly(T=48)
    both(dp, year, store_all=False)


def test_noalloc_rejects_what_it_cannot_hold(dp):
    # 3 planes of 1024 x 4096 floats exceed the 32 MiB array: rejected before device work
    st = wl.random_small(1, 2, 1024, 4096, 3, 3).storage
    lam = torch.zeros(2, 1024, device="cuda")
    P = torch.zeros(2, 1024, 1024, device="cuda")
    V = torch.empty(1024, 4096, device="cuda")
    with pytest.raises(dp.DPError) as e:
        dp.solve_noalloc(lam, P, st, V)
    assert e.value.code == -7 and "dp_solve" in str(e.value)


def test_noalloc_rejects_validation(dp):
    inst = wl.random_small(2, 3, 4, 30, 3, 3)
    lam, P = dev(inst.lam), dev(inst.P)
    pb = dp.make_problem(inst.T, inst.K, inst.storage, dp.DP_VALIDATE)
    import ctypes
    V = torch.empty(inst.K, inst.storage.S, device="cuda")
    rc = dp.lib().dp_solve_noalloc(ctypes.byref(pb), ctypes.c_void_p(lam.data_ptr()),
                                   ctypes.c_void_p(P.data_ptr()), None,
                                   ctypes.c_void_p(V.data_ptr()), None, None, None)
    assert rc == -1 and b"DP_VALIDATE" in dp.lib().dp_last_error()
