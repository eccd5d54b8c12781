"""Batched solves of many heterogeneous instances (binding of dp_batch_*)."""
from __future__ import annotations

import ctypes
from typing import List, Sequence

import torch

from ._lib import check, lib, make_problem


class BatchPlan:
    """A plan for a fixed list of instances (T_i, K_i, storage_i)."""

    def __init__(self, problems: Sequence, tune_cache: str = None, stream=None):
        self.problems = [make_problem(T, K, st) for (T, K, st) in problems]
        n = len(self.problems)
        arr = (type(self.problems[0]) * n)(*self.problems)
        self._arr = arr
        h = ctypes.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream()
        check(lib().dp_batch_plan_create(ctypes.byref(h), n, arr,
                                         tune_cache.encode() if tune_cache else None,
                                         ctypes.c_void_p(s.cuda_stream)))
        self._h = h

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        check(lib().dp_batch_plan_describe(self._h, buf, len(buf)))
        return buf.value.decode()

    def _ptrs(self, tensors):
        n = len(self.problems)
        arr = (ctypes.c_void_p * n)()
        for i, t in enumerate(tensors):
            arr[i] = None if t is None else t.data_ptr()
        return arr

    def _check_io(self, lams, Ps, V1s, policies):
        from . import _check
        n = len(self.problems)
        lists = [("lams", lams), ("Ps", Ps), ("V1s", V1s)] + ([("policies", policies)] if policies is not None else [])
        for name, seq in lists:
            if len(seq) != n:
                raise ValueError(f"{name} must hold {n} tensors, got {len(seq)}")
        dev = lams[0].device
        for i, pb in enumerate(self.problems):
            T, K, S = pb.T, pb.K, pb.st.S
            _check(lams[i], f"lams[{i}]", (T, K), torch.float32, dev)
            _check(Ps[i], f"Ps[{i}]", (T, K, K), torch.float32, dev)
            _check(V1s[i], f"V1s[{i}]", (K, S), torch.float32, dev)
            if policies is not None:
                _check(policies[i], f"policies[{i}]", (T, K, S), torch.int16, dev)

    def solve(self, lams: List[torch.Tensor], Ps: List[torch.Tensor], V1s: List[torch.Tensor],
              policies=None, *, looped: bool = False, graph: bool = True, stream=None):
        """Batched solve (graph replay); graph=False issues the same launches directly;
        looped=True runs one dp_solve per instance instead."""
        from . import _stream
        self._check_io(lams, Ps, V1s, policies)
        s = _stream(stream)
        if looped:
            f = lib().dp_batch_solve_looped
        else:
            f = lib().dp_batch_solve if graph else lib().dp_batch_solve_eager
        pol = self._ptrs(policies) if policies is not None else None
        check(f(self._h, self._ptrs(lams), self._ptrs(Ps), self._ptrs(V1s), pol, s))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dp_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
