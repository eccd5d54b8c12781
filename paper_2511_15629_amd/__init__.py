"""dpgpu: MI355X backward induction for stochastic storage arbitrage (Python binding).

Thin layer over libdpgpu.so (see include/dpgpu.h).  PyTorch supplies device memory
and the current HIP stream; every step of the computation runs in the library's HIP
kernels.

    out = solve(lam, P, storage)                 # V_1 [K, S] float32, policy [T, K, S] int16
    V1 = DPFunction.apply(lam, P, storage, 16)   # differentiable in lam and P
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import DPError, DP_STORE_V_ALL, DP_VALIDATE, check, lib, make_problem

__all__ = ["solve", "solve_noalloc", "adjoint", "Solver", "DPFunction", "DPError",
           "set_sweep_shape",
           "BatchPlan", "kernel_timing", "solve_independent", "power_grid_size"]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    """The HIP stream for a library call.  A stream other than torch's current one first
    waits for the current stream, where the binding made its contiguous copies and
    allocations (and the caller's pending work on the inputs may still run)."""
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cur = torch.cuda.current_stream(stream.device)
    if stream != cur:
        stream.wait_stream(cur)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(x, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return x.contiguous()


def _check(x, name, shape, dtype, device):
    """The library trusts sizes: every array it reads or writes is checked here."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if x.device != device:
        raise ValueError(f"{name} is on {x.device}, expected {device}")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _keep(stream, *tensors):
    """On a stream other than torch's current one, tell the caching allocator that these
    buffers are in use there until the queued work ends."""
    if stream is None:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def set_sweep_shape(tile: int = 0, waves: int = 0):
    """Force the sweep tile shape -- `tile` SoC indices per block on `waves` waves (tuning
    hook); no arguments restores the default."""
    check(lib().dp_set_sweep_shape(tile, waves))


def kernel_timing(on: Optional[bool] = None):
    """With on=True/False switch the library's per-launch event timing; with no argument
    return and reset (sweep_ms, n_sweep, expectation_ms, n_expectation)."""
    L = lib()
    if on is not None:
        check(L.dp_set_timing(1 if on else 0))
        return None
    a, b = ctypes.c_double(), ctypes.c_double()
    na, nb = ctypes.c_int(), ctypes.c_int()
    check(L.dp_get_timing(ctypes.byref(a), ctypes.byref(na), ctypes.byref(b), ctypes.byref(nb)))
    return a.value, na.value, b.value, nb.value


class Solver:
    """Reusable solve: problem record, workspace and outputs allocated once, so repeated
    calls (benchmarks, serving loops) allocate nothing."""

    def __init__(self, lam: torch.Tensor, P: torch.Tensor, storage, *, store_all=False,
                 policy=True, ckpt_every=0):
        self.lam = _dev_f32(lam, "lam")
        self.P = _dev_f32(P, "P")
        T, K = self.lam.shape
        if tuple(self.P.shape) != (T, K, K):
            raise ValueError("P must be [T, K, K]")
        S = int(storage.S)
        self.pb = make_problem(T, K, storage, DP_STORE_V_ALL if store_all else 0, ckpt_every)
        L = lib()
        dev = self.lam.device
        self.V = torch.empty((T + 1, K, S) if store_all else (K, S), dtype=torch.float32,
                             device=dev)
        self.policy = torch.empty((T, K, S), dtype=torch.int16, device=dev) if policy else None
        self.ckpt = _workspace(L.dp_ckpt_bytes(ctypes.byref(self.pb)), dev) if ckpt_every else None
        nws = L.dp_workspace_bytes(ctypes.byref(self.pb))
        if nws == 0:
            check(_lib.DP_EINVAL)
        self.ws = _workspace(nws, dev)

    def run(self, v_term: Optional[torch.Tensor] = None, stream=None):
        if v_term is not None:
            K, S = self.pb.K, self.pb.st.S
            _check(v_term, "v_term", (K, S), torch.float32, self.lam.device)
        check(lib().dp_solve(ctypes.byref(self.pb), _ptr(self.lam), _ptr(self.P), _ptr(v_term),
                             _ptr(self.V), _ptr(self.policy), _ptr(self.ckpt), _ptr(self.ws),
                             ctypes.c_size_t(self.ws.numel()), _stream(stream)))
        return self.V


def solve_noalloc(lam: torch.Tensor, P: torch.Tensor, storage, V: torch.Tensor,
                  policy: Optional[torch.Tensor] = None, v_term: Optional[torch.Tensor] = None,
                  *, store_all: bool = False, ckpt: Optional[torch.Tensor] = None,
                  ckpt_every: int = 0, stream=None) -> torch.Tensor:
    """dp_solve_noalloc: the solve into caller-given outputs (V [T+1, K, S] with store_all,
    else [K, S]; policy [T, K, S] int16 or None), with the solver state in the library's own
    device array, so the call allocates nothing (argument checks only, no copies)."""
    T, K = lam.shape
    S = int(storage.S)
    _check(lam, "lam", (T, K), torch.float32, lam.device)
    _check(P, "P", (T, K, K), torch.float32, lam.device)
    _check(V, "V", (T + 1, K, S) if store_all else (K, S), torch.float32, lam.device)
    if policy is not None:
        _check(policy, "policy", (T, K, S), torch.int16, lam.device)
    if v_term is not None:
        _check(v_term, "v_term", (K, S), torch.float32, lam.device)
    pb = make_problem(T, K, storage, DP_STORE_V_ALL if store_all else 0, ckpt_every)
    if ckpt is not None:
        _check(ckpt, "ckpt", None, torch.uint8, lam.device)
        if ckpt.numel() < lib().dp_ckpt_bytes(ctypes.byref(pb)):
            raise ValueError("ckpt buffer smaller than dp_ckpt_bytes")
    check(lib().dp_solve_noalloc(ctypes.byref(pb), _ptr(lam), _ptr(P), _ptr(v_term), _ptr(V),
                                 _ptr(policy), _ptr(ckpt), _stream(stream)))
    return V


def _iid_problem(T, R, S, delta, eta, p_bar, store_all=False):
    return _lib.IidProblem(int(T), int(R), int(S), 0, float(delta), float(eta), float(p_bar),
                           DP_STORE_V_ALL if store_all else 0)


def power_grid_size(S: int, delta: float, eta: float, p_bar: float):
    """(P, n_c, n_d) of the paper's recombining power grid (host only)."""
    pb = _iid_problem(1, 1, S, delta, eta, p_bar)
    P, nc, nd = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib().dp_iid_action_grid(ctypes.byref(pb), ctypes.byref(P), ctypes.byref(nc),
                                   ctypes.byref(nd)))
    return P.value, nc.value, nd.value


def solve_independent(lam: torch.Tensor, prob: torch.Tensor, S: int, delta: float, eta: float,
                      p_bar: float, *, store_all: bool = False, policy: bool = False,
                      stream=None):
    """Stagewise-independent prices on the paper's power grid (Algorithm 1 as printed).

    lam, prob [T, R] float32 device tensors (sampled levels and their probabilities).
    Returns V ([T+1, S] expected values V_t if store_all, else V_0 [S]) and optionally the
    int16 action index (ascending power grid) per stage, sample and SoC, [T, R, S].
    """
    lam = _dev_f32(lam, "lam")
    prob = _dev_f32(prob, "prob")
    if lam.dim() != 2:
        raise ValueError("lam must be [T, R]")
    T, R = lam.shape
    _check(prob, "prob", (T, R), torch.float32, lam.device)
    pb = _iid_problem(T, R, S, delta, eta, p_bar, store_all)
    L = lib()
    nws = L.dp_iid_workspace_bytes(ctypes.byref(pb))
    if nws == 0:
        check(_lib.DP_EINVAL)
    dev = lam.device
    V = torch.empty((T + 1, S) if store_all else (S,), dtype=torch.float32, device=dev)
    pol = torch.empty((T, R, S), dtype=torch.int16, device=dev) if policy else None
    ws = _workspace(nws, dev)
    check(L.dp_solve_iid(ctypes.byref(pb), _ptr(lam), _ptr(prob), _ptr(V), _ptr(pol), _ptr(ws),
                         ctypes.c_size_t(ws.numel()), _stream(stream)))
    _keep(stream, lam, prob, ws)
    return {"V": V, "policy": pol, "_ws": ws}


def solve(lam: torch.Tensor, P: torch.Tensor, storage, v_term: Optional[torch.Tensor] = None,
          *, store_all: bool = False, policy: bool = True, ckpt_every: int = 0,
          validate: bool = False, stream=None):
    """Backward induction on the GPU.

    lam [T, K], P [T, K, K] float32 device tensors; storage has S, w_up, w_down, delta,
    eta_c, eta_d, c_deg, c_start.  Returns a dict with ``V`` ([T+1, K, S] if store_all
    else V_1 [K, S]), ``policy`` ([T, K, S] int16 or None), ``ckpt`` (uint8 buffer or None)
    and the problem record.
    """
    lam = _dev_f32(lam, "lam")
    P = _dev_f32(P, "P")
    if lam.dim() != 2:
        raise ValueError("lam must be [T, K]")
    T, K = lam.shape
    _check(P, "P", (T, K, K), torch.float32, lam.device)
    S = int(storage.S)
    flags = (DP_STORE_V_ALL if store_all else 0) | (DP_VALIDATE if validate else 0)
    pb = make_problem(T, K, storage, flags, ckpt_every)
    L = lib()
    dev = lam.device
    if v_term is not None:
        v_term = _check(_dev_f32(v_term, "v_term"), "v_term", (K, S), torch.float32, dev)
    V = torch.empty((T + 1, K, S) if store_all else (K, S), dtype=torch.float32, device=dev)
    pol = torch.empty((T, K, S), dtype=torch.int16, device=dev) if policy else None
    ck = None
    if ckpt_every:
        ck = _workspace(L.dp_ckpt_bytes(ctypes.byref(pb)), dev)
    nws = L.dp_workspace_bytes(ctypes.byref(pb))
    if nws == 0:
        check(_lib.DP_EINVAL)
    ws = _workspace(nws, dev)
    check(L.dp_solve(ctypes.byref(pb), _ptr(lam), _ptr(P), _ptr(v_term), _ptr(V), _ptr(pol),
                     _ptr(ck), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(stream)))
    _keep(stream, lam, P, v_term, ws)
    return {"V": V, "policy": pol, "ckpt": ck, "problem": pb, "_ws": ws}


def adjoint(lam, P, storage, seed, *, V_all=None, policy=None, ckpt=None, ckpt_every: int = 0,
            v_term=None, want_vterm: bool = False, validate: bool = False, stream=None):
    """Gradients of J = sum(seed * V_1) w.r.t. lam [T, K], P [T, K, K] (and v_term).
    validate=True checks the rows of P and every given policy entry on the device first."""
    lam = _dev_f32(lam, "lam")
    P = _dev_f32(P, "P")
    seed = _dev_f32(seed, "seed")
    if lam.dim() != 2:
        raise ValueError("lam must be [T, K]")
    T, K = lam.shape
    S = int(storage.S)
    dev = lam.device
    _check(P, "P", (T, K, K), torch.float32, dev)
    _check(seed, "seed", (K, S), torch.float32, dev)
    pb = make_problem(T, K, storage, DP_VALIDATE if validate else 0,
                      ckpt_every if ckpt is not None else 0)
    L = lib()
    if ckpt is not None:
        _check(ckpt, "ckpt", None, torch.uint8, dev)
        if ckpt.numel() < L.dp_ckpt_bytes(ctypes.byref(pb)):
            raise ValueError("ckpt is smaller than dp_ckpt_bytes for this problem")
    if V_all is not None:
        _check(V_all, "V_all", (T + 1, K, S), torch.float32, dev)
    if policy is not None:
        _check(policy, "policy", (T, K, S), torch.int16, dev)
    g_lam = torch.empty((T, K), dtype=torch.float32, device=dev)
    g_P = torch.empty((T, K, K), dtype=torch.float32, device=dev)
    g_v = torch.empty((K, S), dtype=torch.float32, device=dev) if want_vterm else None
    ws = _workspace(L.dp_adjoint_workspace_bytes(ctypes.byref(pb)), dev)
    if v_term is not None:
        v_term = _check(_dev_f32(v_term, "v_term"), "v_term", (K, S), torch.float32, dev)
    check(L.dp_adjoint(ctypes.byref(pb), _ptr(lam), _ptr(P), _ptr(v_term),
                       _ptr(V_all), _ptr(policy), _ptr(ckpt), _ptr(seed), _ptr(g_lam),
                       _ptr(g_P), _ptr(g_v), _ptr(ws), ctypes.c_size_t(ws.numel()),
                       _stream(stream)))
    _keep(stream, lam, P, seed, v_term, ws)
    return {"grad_lam": g_lam, "grad_P": g_P, "grad_vterm": g_v}


class DPFunction(torch.autograd.Function):
    """V_1 = DP(lam, P) with a hand-written adjoint.

    forward(lam [T,K], P [T,K,K], storage, ckpt_every=0) -> V_1 [K, S].
    ckpt_every = 0 keeps all stage values and int16 policies for the backward pass;
    ckpt_every = n keeps value checkpoints every n stages and recomputes each segment's
    values and policies in backward (bitwise the same as the forward pass).
    The gradient is exact for the fixed argmax policies (almost everywhere).
    """

    @staticmethod
    def forward(ctx, lam, P, storage, ckpt_every: int = 0):
        if ckpt_every:
            out = solve(lam, P, storage, store_all=False, policy=False, ckpt_every=ckpt_every)
            ctx.save_for_backward(lam, P, out["ckpt"])
        else:
            out = solve(lam, P, storage, store_all=True, policy=True)
            ctx.save_for_backward(lam, P, out["V"], out["policy"])
        ctx.storage = storage
        ctx.ckpt_every = ckpt_every
        return out["V"][0].clone() if not ckpt_every else out["V"]

    @staticmethod
    def backward(ctx, grad_V1):
        seed = grad_V1.contiguous().to(torch.float32)
        if ctx.ckpt_every:
            lam, P, ck = ctx.saved_tensors
            g = adjoint(lam, P, ctx.storage, seed, ckpt=ck, ckpt_every=ctx.ckpt_every)
        else:
            lam, P, V_all, pol = ctx.saved_tensors
            g = adjoint(lam, P, ctx.storage, seed, V_all=V_all, policy=pol)
        return g["grad_lam"], g["grad_P"], None, None


from .batch import BatchPlan  # noqa: E402
