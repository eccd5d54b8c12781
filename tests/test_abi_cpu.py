"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol include/dpgpu.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpgpu.h")


@pytest.fixture(scope="module")
def L():
    from paper_2511_15629_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2511_15629_amd import build
        build.build()
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(dp_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_binding_exports():
    from paper_2511_15629_amd import _lib
    assert set(declared_functions()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_layout_matches_header(L):
    from paper_2511_15629_amd import _lib
    assert ctypes.sizeof(_lib.Storage) == 36
    assert ctypes.sizeof(_lib.Problem) == 52
    assert L.dp_abi_version() == 1


def _pb(**kw):
    from paper_2511_15629_amd import _lib
    import workloads as wl
    st = wl.Storage(S=kw.pop("S", 11), w_up=kw.pop("w_up", 2), w_down=kw.pop("w_down", 2),
                    delta=kw.pop("delta", 0.1), eta_c=kw.pop("eta_c", 0.9),
                    eta_d=kw.pop("eta_d", 0.9), c_deg=kw.pop("c_deg", 1.0),
                    c_start=kw.pop("c_start", 0.0))
    return _lib.make_problem(kw.pop("T", 4), kw.pop("K", 3), st, kw.pop("flags", 0),
                             kw.pop("ckpt_every", 0))


@pytest.mark.parametrize("bad", [dict(T=0), dict(K=0), dict(K=5000), dict(S=1),
                                 dict(S=40000), dict(w_up=-1), dict(delta=0.0),
                                 dict(eta_c=1.5), dict(eta_d=0.0), dict(c_deg=-1.0),
                                 dict(c_start=float("nan")), dict(flags=0x80),
                                 dict(ckpt_every=-2)])
def test_invalid_problems_are_rejected_on_the_host(L, bad):
    pb = _pb(**bad)
    assert L.dp_workspace_bytes(ctypes.byref(pb)) == 0
    assert L.dp_last_error()
    rc = L.dp_solve(ctypes.byref(pb), 1, 1, None, 1, None, None, 256, 1 << 20, None)
    assert rc == -1


def test_missing_pointers_and_small_workspace(L):
    pb = _pb()
    need = L.dp_workspace_bytes(ctypes.byref(pb))
    assert need > 0
    assert L.dp_solve(ctypes.byref(pb), None, 1, None, 1, None, None, 256, need, None) == -1
    assert L.dp_solve(ctypes.byref(pb), 1, 1, None, 1, None, None, 256, need - 1, None) == -3
    assert L.dp_solve(ctypes.byref(pb), 1, 1, None, 1, None, None, 0x1001, need, None) == -1
    assert b"aligned" in L.dp_last_error()
    assert L.dp_strerror(-3) == b"workspace missing or too small"


def test_adjoint_argument_rules(L):
    pb = _pb(ckpt_every=4)
    need = L.dp_adjoint_workspace_bytes(ctypes.byref(pb))
    assert need > 0
    # both full-storage inputs and a checkpoint: rejected
    rc = L.dp_adjoint(ctypes.byref(pb), 1, 1, None, 1, 1, 1, 1, 1, 1, None, 256, need, None)
    assert rc == -1
    # every S up to DP_MAX_S is accepted (the push-forward takes the next states in
    # chunks); a too-small workspace is still rejected before any device work
    pb2 = _pb(S=32767)
    need2 = L.dp_adjoint_workspace_bytes(ctypes.byref(pb2))
    assert need2 > 0
    rc = L.dp_adjoint(ctypes.byref(pb2), 1, 1, None, 1, 1, None, 1, 1, 1, None, 256, need2 - 1, None)
    assert rc == -3


def test_checkpoint_size_counts_interior_slots(L):
    pb = _pb(T=288, K=100, S=1001, ckpt_every=16)
    n = L.dp_ckpt_bytes(ctypes.byref(pb))
    slots = (288 - 1) // 16
    assert n >= slots * 100 * 1001 * 4 + slots * 8
    assert n < (slots + 1) * 100 * 1001 * 4 + 4096


def _iid(**kw):
    from paper_2511_15629_amd import _lib
    f = dict(T=4, R=5, S=41, reserved=0, delta=0.1, eta=0.9219544, p_bar=1.0, flags=0)
    f.update(kw)
    return _lib.IidProblem(**f)


def test_iid_struct_and_action_grid_match_the_paper(L):
    # P counts of Table 1 at eta = sqrt(0.85), p_bar = 1 (tests/golden/grid_counts.txt)
    from paper_2511_15629_amd import _lib
    assert ctypes.sizeof(_lib.IidProblem) == 32
    golden = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "grid_counts.txt")):
        parts = line.split()
        if parts and parts[0] == "P":
            golden[float(parts[1])] = int(parts[3])
    for delta, want in golden.items():
        pb = _iid(delta=delta)
        P, nc, nd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        assert L.dp_iid_action_grid(ctypes.byref(pb), ctypes.byref(P), ctypes.byref(nc),
                                    ctypes.byref(nd)) == 0
        assert P.value == want and nc.value + nd.value + 1 == want


@pytest.mark.parametrize("bad", [dict(T=0), dict(R=0), dict(R=5000), dict(S=1), dict(S=40000),
                                 dict(delta=0.0), dict(eta=1.5), dict(eta=0.0), dict(p_bar=0.0),
                                 dict(p_bar=float("inf")), dict(flags=0x2), dict(reserved=1),
                                 dict(delta=1e-5)])
def test_invalid_iid_problems_are_rejected_on_the_host(L, bad):
    pb = _iid(**bad)
    assert L.dp_iid_workspace_bytes(ctypes.byref(pb)) == 0
    rc = L.dp_solve_iid(ctypes.byref(pb), 1, 1, 1, None, 256, 1 << 20, None)
    assert rc in (-1, -7)
    assert L.dp_last_error()


def test_iid_lds_limit_and_workspace_rules(L):
    # R = 4096 samples over a 32767-level grid need more LDS per block than a CU holds
    pb = _iid(R=4096, S=32767, delta=0.01)
    assert L.dp_solve_iid(ctypes.byref(pb), 1, 1, 1, None, 256, 1 << 30, None) == -7
    pb = _iid()
    need = L.dp_iid_workspace_bytes(ctypes.byref(pb))
    assert need > 0
    assert L.dp_solve_iid(ctypes.byref(pb), None, 1, 1, None, 256, need, None) == -1
    assert L.dp_solve_iid(ctypes.byref(pb), 1, 1, 1, None, 256, need - 1, None) == -3
    assert L.dp_solve_iid(ctypes.byref(pb), 1, 1, 1, None, 0x1001, need, None) == -1


def test_windows_beyond_lds_are_rejected_before_device_work(L):
    # the smallest tile (64 outputs, one wave) holds, per side, the u array over 63 + w next
    # states (rounded up to 8) and two tables of 80 16-bit positions, the expectation row
    # over 64 + w_up + w_down next states and row k of P_t (K = 3, padded to 8) in 160 KiB:
    # up to +-10148, not +-10149
    pb = _pb(S=32767, w_up=10149, w_down=10149)
    assert L.dp_workspace_bytes(ctypes.byref(pb)) == 0
    assert L.dp_solve(ctypes.byref(pb), 1, 1, None, 1, None, None, 256, 1 << 30, None) == -7
    assert b"LDS" in L.dp_last_error()
    pb = _pb(S=32767, w_up=10148, w_down=10148)
    assert L.dp_workspace_bytes(ctypes.byref(pb)) > 0
