"""FP64 CPU oracle for the storage-arbitrage DP.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It shares no code with the HIP path (``paper_2511_15629_amd``)
and imports nothing from it; the only common dependency is the seeded input generator
module ``workloads``, which holds no DP arithmetic.

Contents
--------
* ``solve``, ``stage``, ``adjoint``, ``policy_value`` -- plain C loops in FP64
  (``dp_oracle.c``), the definition of the backward induction of Eq. (5)-(6) on the
  integer action window of Sec. III (recombining grid) with a Markov price chain.
* ``brute`` -- exhaustive enumeration of non-anticipative plans on tiny scenario trees.
* ``lp`` -- the deterministic arbitrage LP of Eq. (1) with separate charge/discharge
  (SciPy HiGHS), an upper bound on the DP and equal to it in the TU special case.
* ``alg1`` -- Algorithm 1 of the paper written out with NumPy array operations for the
  stagewise-independent model (power-action grid, interpolation, -inf mask, max, mean).
* ``hull`` -- the concave envelope of a finite point set by its definition (max over
  pairs), used to check the host bid-curve convexifier (Eq. (9)-(10)).
* ``arbitrage`` -- the continuous deterministic problem of Eq. (1)-(2) as the MILP of
  Eq. (3a)-(3d), its LP relaxation, the LP restriction of Sec. V-B and the plain LP
  (SciPy HiGHS, sparse), for the accuracy studies of Sec. V.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile dp_oracle.c with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", _LIB + ".tmp",
               _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            i, d, p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
            lib.oracle_stage.argtypes = [i, i, i, i, d, d, d, d, d, p, p, p, p, p, p, i]
            lib.oracle_solve.argtypes = [i, i, i, i, i, d, d, d, d, d, p, p, p, p, p, p, i]
            lib.oracle_adjoint.argtypes = [i, i, i, i, i, d, d, d, d, d, p, p, p, p, p, p, p, p, i]
            lib.oracle_policy_value.argtypes = [i, i, i, i, i, d, d, d, d, d, p, p, p, p, p]
            lib.oracle_max_threads.argtypes = []
            for f in (lib.oracle_stage, lib.oracle_solve, lib.oracle_adjoint,
                      lib.oracle_policy_value, lib.oracle_max_threads):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _st(st):
    return (int(st.S), int(st.w_up), int(st.w_down), float(st.delta), float(st.eta_c),
            float(st.eta_d), float(st.c_deg), float(st.c_start))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def stage(st, lam_t, P_t, v_next, *, want_w: bool = False, threads: int = 0):
    """One Bellman stage from FP64 V_{t+1} [K, S]; returns (V_t, pi_t[, W_t])."""
    lib = _load()
    lam_t, P_t = _f32(lam_t), _f32(P_t)
    K = lam_t.shape[0]
    vn = np.ascontiguousarray(v_next, dtype=np.float64)
    assert vn.shape == (K, st.S) and P_t.shape == (K, K)
    Vt = np.empty((K, st.S), np.float64)
    pol = np.empty((K, st.S), np.int16)
    W = np.empty((K, st.S), np.float64) if want_w else None
    S, wu, wd, de, ec, ed, cd, cs = _st(st)
    lib.oracle_stage(K, S, wu, wd, de, ec, ed, cd, cs, _ptr(lam_t), _ptr(P_t), _ptr(vn),
                     _ptr(W), _ptr(Vt), _ptr(pol), int(threads))
    return (Vt, pol, W) if want_w else (Vt, pol)


def solve(st, lam, P, v_term=None, *, keep_all: bool = True, want_policy: bool = True,
          threads: int = 0):
    """Backward induction t = T..1.  Returns dict with V1 [K,S], V [T+1,K,S] (if
    keep_all), policy [T,K,S] int16 (if want_policy)."""
    lib = _load()
    lam, P = _f32(lam), _f32(P)
    T, K = lam.shape
    assert P.shape == (T, K, K)
    S = st.S
    vt = None if v_term is None else np.ascontiguousarray(v_term, dtype=np.float64)
    V_all = np.empty((T + 1, K, S), np.float64) if keep_all else None
    V1 = np.empty((K, S), np.float64)
    pol = np.empty((T, K, S), np.int16) if want_policy else None
    S_, wu, wd, de, ec, ed, cd, cs = _st(st)
    rc = lib.oracle_solve(T, K, S_, wu, wd, de, ec, ed, cd, cs, _ptr(lam), _ptr(P), _ptr(vt),
                          _ptr(V_all), _ptr(V1), _ptr(pol), int(threads))
    if rc != 0:
        raise MemoryError("oracle_solve failed")
    return {"V1": V1, "V": V_all, "policy": pol}


def adjoint(st, lam, P, V_all, policy, seed, *, threads: int = 0):
    """Gradients of J = sum(seed * V_1) for fixed policies (FP64)."""
    lib = _load()
    lam, P = _f32(lam), _f32(P)
    T, K = lam.shape
    S = st.S
    V_all = np.ascontiguousarray(V_all, dtype=np.float64)
    policy = np.ascontiguousarray(policy, dtype=np.int16)
    seed = np.ascontiguousarray(seed, dtype=np.float64)
    assert V_all.shape == (T + 1, K, S) and policy.shape == (T, K, S) and seed.shape == (K, S)
    gl = np.empty((T, K), np.float64)
    gP = np.empty((T, K, K), np.float64)
    gv = np.empty((K, S), np.float64)
    S_, wu, wd, de, ec, ed, cd, cs = _st(st)
    rc = lib.oracle_adjoint(T, K, S_, wu, wd, de, ec, ed, cd, cs, _ptr(lam), _ptr(P),
                            _ptr(V_all), _ptr(policy), _ptr(seed), _ptr(gl), _ptr(gP),
                            _ptr(gv), int(threads))
    if rc != 0:
        raise MemoryError("oracle_adjoint failed")
    return {"grad_lam": gl, "grad_P": gP, "grad_vterm": gv}


def policy_value(st, lam, P, policy, v_term=None):
    """V_1 of a fixed policy set by backward evaluation (no maximisation)."""
    lib = _load()
    lam, P = _f32(lam), _f32(P)
    T, K = lam.shape
    vt = None if v_term is None else np.ascontiguousarray(v_term, dtype=np.float64)
    policy = np.ascontiguousarray(policy, dtype=np.int16)
    V1 = np.empty((K, st.S), np.float64)
    S_, wu, wd, de, ec, ed, cd, cs = _st(st)
    lib.oracle_policy_value(T, K, S_, wu, wd, de, ec, ed, cd, cs, _ptr(lam), _ptr(P),
                            _ptr(vt), _ptr(policy), _ptr(V1))
    return V1


def q_values(st, lam_t_k: float, w_row: np.ndarray, s: int) -> np.ndarray:
    """Q(s, j) = r(lambda, j - s) + W[j] for every feasible j (FP64), as a dict-like array
    indexed by j (entries outside J(s) are -inf)."""
    S = st.S
    q = np.full(S, -np.inf)
    lo, hi = max(0, s - st.w_down), min(S - 1, s + st.w_up)
    for j in range(lo, hi + 1):
        d = j - s
        if d > 0:
            g = -d * st.delta / st.eta_c
        elif d < 0:
            g = -d * st.delta * st.eta_d
        else:
            g = 0.0
        q[j] = lam_t_k * g - st.c_deg * abs(g) - (st.c_start if d != 0 else 0.0) + w_row[j]
    return q


def q_at(st, lam_t, W, k, s, j) -> np.ndarray:
    """Q(k, s, j) = r(lambda_t[k], j - s) + W[k][j] for index arrays k, s, j (FP64; -inf
    where j is outside J(s)): the candidate values of given (state, move) pairs, for
    checking a chosen move against the maximum."""
    k, s, j = (np.asarray(a, dtype=np.int64) for a in (k, s, j))
    d = j - s
    dd = d.astype(np.float64)
    g = np.where(d > 0, -dd * st.delta / st.eta_c, np.where(d < 0, -dd * st.delta * st.eta_d, 0.0))
    lam = np.asarray(lam_t, dtype=np.float64)[k]
    r = lam * g - st.c_deg * np.abs(g) - np.where(d != 0, st.c_start, 0.0)
    ok = (j >= np.maximum(0, s - st.w_down)) & (j <= np.minimum(st.S - 1, s + st.w_up))
    wv = np.asarray(W, dtype=np.float64)[k, np.clip(j, 0, st.S - 1)]
    return np.where(ok, r + wv, -np.inf)
