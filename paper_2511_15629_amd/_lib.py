"""ctypes view of libdpgpu.so (the C ABI declared in include/dpgpu.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of the
library.  If the shared library is missing the import fails loudly; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpgpu.so")

DP_OK = 0
DP_EINVAL = -1
DP_EBADPROB = -2
DP_ENOWS = -3
DP_EHIP = -4
DP_ETIMEOUT = -5
DP_ENOMEM = -6
DP_ENOTSUP = -7

DP_STORE_V_ALL = 0x1
DP_VALIDATE = 0x2

# Every symbol include/dpgpu.h declares (the tests check the library exports all of them).
EXPORTS = (
    "dp_abi_version", "dp_strerror", "dp_last_error", "dp_workspace_bytes", "dp_ckpt_bytes",
    "dp_solve", "dp_solve_noalloc", "dp_adjoint_workspace_bytes", "dp_adjoint", "dp_batch_plan_create",
    "dp_batch_solve", "dp_batch_solve_eager", "dp_batch_solve_looped", "dp_batch_plan_describe",
    "dp_batch_plan_destroy", "dp_set_sweep_shape", "dp_set_timing", "dp_get_timing",
    "dp_iid_action_grid", "dp_iid_workspace_bytes", "dp_solve_iid",
)


class DPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dpgpu error {code}: {msg}")
        self.code = code


class Storage(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("w_up", ctypes.c_int32), ("w_down", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("delta", ctypes.c_float),
                ("eta_c", ctypes.c_float), ("eta_d", ctypes.c_float),
                ("c_deg", ctypes.c_float), ("c_start", ctypes.c_float)]


class IidProblem(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("R", ctypes.c_int32), ("S", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("delta", ctypes.c_float), ("eta", ctypes.c_float),
                ("p_bar", ctypes.c_float), ("flags", ctypes.c_uint32)]


class Problem(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("K", ctypes.c_int32), ("st", Storage),
                ("flags", ctypes.c_uint32), ("ckpt_every", ctypes.c_int32)]


_lib = None


def lib():
    """Load libdpgpu.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2511_15629_amd.build` "
                "(hipcc, gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        p, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        PP = ctypes.POINTER(Problem)
        sig = {
            "dp_abi_version": ([], i),
            "dp_strerror": ([i], ctypes.c_char_p),
            "dp_last_error": ([], ctypes.c_char_p),
            "dp_workspace_bytes": ([PP], sz),
            "dp_ckpt_bytes": ([PP], sz),
            "dp_solve": ([PP, p, p, p, p, p, p, p, sz, p], i),
            "dp_solve_noalloc": ([PP, p, p, p, p, p, p, p], i),
            "dp_adjoint_workspace_bytes": ([PP], sz),
            "dp_adjoint": ([PP, p, p, p, p, p, p, p, p, p, p, p, sz, p], i),
            "dp_batch_plan_create": ([ctypes.POINTER(p), i, PP, ctypes.c_char_p, p], i),
            "dp_batch_solve": ([p, p, p, p, p, p], i),
            "dp_batch_solve_eager": ([p, p, p, p, p, p], i),
            "dp_batch_solve_looped": ([p, p, p, p, p, p], i),
            "dp_batch_plan_describe": ([p, ctypes.c_char_p, sz], i),
            "dp_batch_plan_destroy": ([p], None),
            "dp_set_sweep_shape": ([i, i], i),
            "dp_set_timing": ([i], i),
            "dp_iid_action_grid": ([ctypes.POINTER(IidProblem), ctypes.POINTER(i),
                                    ctypes.POINTER(i), ctypes.POINTER(i)], i),
            "dp_iid_workspace_bytes": ([ctypes.POINTER(IidProblem)], sz),
            "dp_solve_iid": ([ctypes.POINTER(IidProblem), p, p, p, p, p, sz, p], i),
            "dp_get_timing": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)], i),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc: int):
    if rc != DP_OK:
        L = lib()
        raise DPError(rc, f"{L.dp_strerror(rc).decode()}: {L.dp_last_error().decode()}")
    return rc


def make_problem(T: int, K: int, storage, flags: int = 0, ckpt_every: int = 0) -> Problem:
    st = Storage(int(storage.S), int(storage.w_up), int(storage.w_down), 0,
                 float(storage.delta), float(storage.eta_c), float(storage.eta_d),
                 float(getattr(storage, "c_deg", 0.0)), float(getattr(storage, "c_start", 0.0)))
    return Problem(int(T), int(K), st, int(flags), int(ckpt_every))
