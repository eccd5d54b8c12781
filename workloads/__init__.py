"""Seeded synthetic inputs for the storage-arbitrage DP (price chains and storage sets).

This module only *generates inputs*: price levels lambda_t[k], Markov transition
matrices P_t[k, k'] and storage parameters.  It holds none of the DP arithmetic
(no payoff, no Bellman step, no expectation), so both the FP64 oracle and the HIP
path may consume it.

The paper (Sec. IV "Data") builds 200-sample quantile forecasts from ISO-NE prices;
that data is not available, so the chains below are synthetic stand-ins with the
shapes of the configurations the paper and its Table 3 use:

* nodes x_k = Phi^-1((k + 1/2) / K) of a latent standard normal on equal-mass bins
  with edges e_k = Phi^-1(k / K);
* a latent AR(1) z_{t+1} = m_{t+1} + rho (z_t - m_t) + sigma_eps eps with a daily
  sinusoidal mean m_t and sigma_eps = sqrt(1 - rho^2) (Tauchen 1986 discretisation);
* levels lambda_t[k] = exp(mu + sigma x_k) - 10 plus N(0, 1) jitter, rounded to FP32;
* P_t quantised to multiples of 2^-24 with exact unit row sums, so that every entry
  and every row sum is exact both in FP32 and in FP64.

All arrays are float32 (the precision both sides consume); FP64 users upcast exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
from scipy.special import ndtr, ndtri

Q24 = float(2 ** 24)


@dataclasses.dataclass(frozen=True)
class Storage:
    """Battery parameters on the SoC grid (Sec. III-A "Discretization").

    S        number of SoC grid points, s_hat = [0, delta, ..., (S-1) delta]
    w_up     W_c: largest upward SoC move per stage (grid steps, charging)
    w_down   W_d: largest downward SoC move per stage (grid steps, discharging)
    delta    MWh per grid step
    eta_c    charging efficiency (grid -> cell), eta_d discharging efficiency
    c_deg    $/MWh on grid-side throughput |g|
    c_start  $ per non-idle stage (non-concave payoff term)
    """

    S: int
    w_up: int
    w_down: int
    delta: float
    eta_c: float
    eta_d: float
    c_deg: float = 0.0
    c_start: float = 0.0

    def as_f32(self) -> "Storage":
        f = lambda x: float(np.float32(x))
        return dataclasses.replace(self, delta=f(self.delta), eta_c=f(self.eta_c),
                                   eta_d=f(self.eta_d), c_deg=f(self.c_deg),
                                   c_start=f(self.c_start))


@dataclasses.dataclass
class Instance:
    """One DP instance: T stages, K price states, storage, lam [T, K], P [T, K, K]."""

    name: str
    T: int
    K: int
    storage: Storage
    lam: np.ndarray          # float32 [T, K]
    P: np.ndarray            # float32 [T, K, K], row k = from-state, rows sum to 1 exactly

    def candidates(self) -> int:
        """Feasible (t, k, s, j) state-action pairs of the whole solve."""
        st = self.storage
        per_k = 0
        S, wu, wd = st.S, st.w_up, st.w_down
        # sum over s of |[max(0, s - wd), min(S - 1, s + wu)]|
        s = np.arange(S, dtype=np.int64)
        per_k = int(np.sum(np.minimum(S - 1, s + wu) - np.maximum(0, s - wd) + 1))
        return per_k * self.K * self.T


def tauchen_nodes(K: int):
    """Equal-mass nodes and bin edges of a standard normal."""
    u = (np.arange(K, dtype=np.float64) + 0.5) / K
    x = ndtri(u)
    e = np.empty(K + 1, dtype=np.float64)
    e[0], e[K] = -np.inf, np.inf
    e[1:K] = ndtri(np.arange(1, K, dtype=np.float64) / K)
    return x, e


def tauchen_transitions(K: int, T: int, rho: float, mean: np.ndarray) -> np.ndarray:
    """FP64 Tauchen transitions P_t, t = 1..T, for a latent AR(1) with mean m_t.

    ``mean`` has length T + 1 (m_1 .. m_{T+1}); P_t links stage t to stage t + 1.
    """
    x, e = tauchen_nodes(K)
    sig = math.sqrt(1.0 - rho * rho)
    P = np.empty((T, K, K), dtype=np.float64)
    for t in range(T):
        mu = mean[t + 1] + rho * (x - mean[t])            # conditional mean, per from-state
        cdf = ndtr((e[None, :] - mu[:, None]) / sig)       # [K, K+1]
        P[t] = np.diff(cdf, axis=1)
    return P


def quantize_rows(P: np.ndarray) -> np.ndarray:
    """Round rows to multiples of 2^-24 with an exact unit sum; return float32.

    Every entry is an integer multiple of 2^-24 in [0, 1] and so exactly
    representable in FP32; the integer numerators of each row add up to 2^24.
    """
    n = np.rint(np.asarray(P, dtype=np.float64) * Q24).astype(np.int64)
    n = np.maximum(n, 0)
    short = (1 << 24) - n.sum(axis=-1)
    flat = n.reshape(-1, n.shape[-1])
    idx = np.argmax(flat, axis=-1)
    flat[np.arange(flat.shape[0]), idx] += short.reshape(-1)
    if np.any(flat < 0):
        raise ValueError("row quantisation produced a negative entry")
    out = (flat.astype(np.float64) / Q24).astype(np.float32).reshape(P.shape)
    return out


def unnormalised_rows(P: np.ndarray, rel: float, *, seed: int) -> np.ndarray:
    """Rows of P scaled by independent factors 1 + U(-rel, rel), rounded to FP32: rows
    that no longer sum to 1 exactly (as estimated or float-rounded transition matrices
    do), for checking that a solver does not rely on exact unit row sums."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fac = 1.0 + rng.uniform(-rel, rel, size=P.shape[:-1] + (1,))
    return f32(np.asarray(P, dtype=np.float64) * fac)


def f32(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def lognormal_levels(x: np.ndarray, mu, sigma: float, shift: float = -10.0) -> np.ndarray:
    """exp(mu + sigma x) + shift, broadcasting mu over stages."""
    return np.exp(np.asarray(mu, dtype=np.float64)[..., None] + sigma * x[None, :]) + shift


def daily_mean(T: int, n_day: int, amp: float = 0.5) -> np.ndarray:
    t = np.arange(1, T + 2, dtype=np.float64)
    return amp * np.sin(2.0 * np.pi * t / n_day)


def markov_chain(T: int, K: int, *, seed: int, n_day: int, rho: float = 0.8,
                 mu: float = 3.5, sigma: float = 0.5, neg_nodes: int = 0,
                 neg_low: float = -150.0, neg_high: float = -5.0):
    """Levels [T, K] (float32) and quantised transitions [T, K, K] (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, _ = tauchen_nodes(K)
    P = quantize_rows(tauchen_transitions(K, T, rho, daily_mean(T, n_day)))
    lam = lognormal_levels(x, np.full(T, mu), sigma)
    if neg_nodes:
        lam[:, :neg_nodes] = np.linspace(neg_low, neg_high, neg_nodes)[None, :]
    lam = lam + rng.standard_normal((T, K))
    return f32(lam), P


def spike_chain(T: int, K_base: int, *, seed: int, n_day: int = 24, rho: float = 0.8,
                p_spike: float = 0.01, spike_mult: float = 10.0, season_amp: float = 0.3):
    """Two-regime chain (base x spike) with seasonal drift of the level mean.

    State index = regime * K_base + node.  The regime is i.i.d. with spike
    probability p_spike; spike levels are spike_mult times the base levels.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    x, _ = tauchen_nodes(K_base)
    Pb = tauchen_transitions(K_base, T, rho, daily_mean(T, n_day))
    R = np.array([[1.0 - p_spike, p_spike], [1.0 - p_spike, p_spike]])
    P = quantize_rows(np.einsum("ab,tij->taibj", R, Pb).reshape(T, 2 * K_base, 2 * K_base))
    t = np.arange(1, T + 1, dtype=np.float64)
    mu = 3.5 + season_amp * np.sin(2.0 * np.pi * t / 8760.0)
    base = lognormal_levels(x, mu, 0.5)
    lam = np.concatenate([base, spike_mult * base], axis=1)
    lam = lam + rng.standard_normal((T, 2 * K_base))
    return f32(lam), P


# ----------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------

def day_hourly_small() -> Instance:
    """T=24 hourly, K=10, 1 MW / 4 MWh, S=101 (delta=0.04), +-25 steps, eta=0.95, c_deg=2."""
    lam, P = markov_chain(24, 10, seed=1, n_day=24)
    st = Storage(S=101, w_up=25, w_down=25, delta=0.04, eta_c=0.95, eta_d=0.95,
                 c_deg=2.0).as_f32()
    return Instance("plain_T24_K10_S101_w25", 24, 10, st, lam, P)


def day_5min(T: int = 288) -> Instance:
    """T=288 five-minute, K=100 (5 lowest nodes at -150..-5 $/MWh), S=1001, +-250, c_deg=2."""
    lam, P = markov_chain(T, 100, seed=2, n_day=288, neg_nodes=5)
    st = Storage(S=1001, w_up=250, w_down=250, delta=0.004, eta_c=0.95, eta_d=0.95,
                 c_deg=2.0).as_f32()
    return Instance(f"plain_T{T}_K100_S1001_w250", T, 100, st, lam, P)


def year_hourly(T: int = 8760) -> Instance:
    """T=8760 hourly, K=50 (2 regimes x 25), S=2001, +-500, start cost 5 $."""
    lam, P = spike_chain(T, 25, seed=3)
    st = Storage(S=2001, w_up=500, w_down=500, delta=0.002, eta_c=0.95, eta_d=0.95,
                 c_deg=0.0, c_start=5.0).as_f32()
    return Instance(f"year_T{T}_K50_S2001_w500_start5", T, 50, st, lam, P)


def day_5min_adjoint() -> Instance:
    inst = day_5min()
    inst.name = "adjoint_T288_K100_S1001_w250"
    return inst


def fd_sub_5min() -> Instance:
    """K=10, S=101, +-25, T=288 sub-instance for finite differences."""
    lam, P = markov_chain(288, 10, seed=5, n_day=288)
    st = Storage(S=101, w_up=25, w_down=25, delta=0.04, eta_c=0.95, eta_d=0.95,
                 c_deg=2.0).as_f32()
    return Instance("adjoint_fd_T288_K10_S101_w25", 288, 10, st, lam, P)


def fleet_5min(n: int = 512, seed: int = 4, T: int = 288, s_max: int = 2001,
             ks: Sequence[int] = (20, 50, 100)) -> List[Instance]:
    """Heterogeneous batch: K in {20,50,100}, S ~ U{201..s_max}, 1-8 h, eta ~ U[0.85,0.98].

    Windows follow a 1 MW rating over 5-minute stages:
    W_c = floor(p dt eta / delta), W_d = floor(p dt / (eta delta)), both >= 1.
    Instances with the same K share one transition tensor (one market, many batteries);
    levels carry per-instance jitter.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    chains = {}
    for K in ks:
        chains[K] = markov_chain(T, K, seed=1000 + K, n_day=288, neg_nodes=max(1, K // 20))
    out = []
    dt = 1.0 / 12.0
    for i in range(n):
        K = int(rng.choice(np.asarray(ks)))
        S = int(rng.integers(201, s_max + 1))
        dur = int(rng.integers(1, 9))
        eta = float(np.float32(rng.uniform(0.85, 0.98)))
        delta = float(np.float32(dur / (S - 1)))
        w_up = max(1, int(math.floor(dt * eta / delta)))
        w_down = max(1, int(math.floor(dt / (eta * delta))))
        w_up, w_down = min(w_up, S - 1), min(w_down, S - 1)
        lam0, P = chains[K]
        lam = f32(lam0.astype(np.float64) + rng.standard_normal(lam0.shape))
        st = Storage(S=S, w_up=w_up, w_down=w_down, delta=delta, eta_c=eta, eta_d=eta,
                     c_deg=2.0).as_f32()
        out.append(Instance(f"batch{i}_K{K}_S{S}_d{dur}", T, K, st, lam, P))
    return out


def random_small(seed: int, T: int, K: int, S: int, w_up: int, w_down: int, *,
                 eta: float = 0.9, c_deg: float = 1.0, c_start: float = 0.0,
                 delta: float = 0.25, lam_lo: float = -20.0, lam_hi: float = 80.0,
                 dirichlet: float = 1.0) -> Instance:
    """Small random instance with arbitrary (Dirichlet) stochastic rows; for pins and parity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = f32(rng.uniform(lam_lo, lam_hi, size=(T, K)))
    P = quantize_rows(rng.dirichlet(np.full(K, dirichlet), size=(T, K)))
    st = Storage(S=S, w_up=w_up, w_down=w_down, delta=delta, eta_c=eta, eta_d=eta,
                 c_deg=c_deg, c_start=c_start).as_f32()
    return Instance(f"rand{seed}_T{T}_K{K}_S{S}", T, K, st, lam, P)


def default_seed(K: int, S: int, s0: int = 0) -> np.ndarray:
    """Objective weights Omega [K, S]: mass 1/K on SoC index s0 for every price state."""
    om = np.zeros((K, S), dtype=np.float32)
    om[:, s0] = np.float32(1.0 / K)
    return om


# ----------------------------------------------------------------------------------
# Stagewise-independent workload shaped like Table 3 (8784 hours, 200 samples per hour)
# ----------------------------------------------------------------------------------

TABLE3 = [(4, 0.1), (20, 0.1), (100, 0.1), (4, 0.01), (20, 0.01), (100, 0.01)]   # (hours, delta)


@dataclasses.dataclass
class IidInstance:
    """Stagewise-independent prices: lam [T, R] levels, prob [T, R] probabilities."""

    name: str
    T: int
    R: int
    S: int
    delta: float
    eta: float
    p_bar: float
    lam: np.ndarray
    prob: np.ndarray


def iid_prices(T: int, R: int, *, seed: int, scale: float = 12.0, dof: float = 3.0):
    """Synthetic hourly day-ahead curve plus R equal-mass quantiles of a heavy-tailed
    real-time spread (Student t), the shape of the quantile forecasts of Sec. IV."""
    from scipy.stats import t as student_t
    rng = np.random.Generator(np.random.PCG64(seed))
    da, h = _day_ahead(T, rng)
    q = student_t.ppf((np.arange(R) + 0.5) / R, dof)
    spread = scale * (1.0 + 0.3 * np.sin(2 * np.pi * h / 24.0))[:, None] * q[None, :]
    lam = f32(da[:, None] + spread)
    prob = quantize_rows(np.full((T, R), 1.0 / R))
    return lam, prob


def _day_ahead(T: int, rng):
    """Hourly day-ahead curve: a daily and a yearly cycle plus Gaussian noise."""
    h = np.arange(T) % 24
    d = np.arange(T) // 24
    da = 45.0 + 15.0 * np.sin(2 * np.pi * (h - 8) / 24.0) + 10.0 * np.sin(2 * np.pi * d / 366.0)
    return da + rng.normal(0.0, 5.0, T), h


def realized_prices(T: int, *, seed: int, scale: float = 12.0, dof: float = 3.0):
    """One realised hourly real-time path [T] (FP32): the day-ahead curve of iid_prices
    plus one Student-t draw of the spread (the perfect-foresight input of Sec. V-A)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    da, h = _day_ahead(T, rng)
    spread = scale * (1.0 + 0.3 * np.sin(2 * np.pi * h / 24.0)) * rng.standard_t(dof, T)
    return f32(da + spread)


def negative_prices(lam):
    """lam - max(lam) (<= 0 everywhere, the level shift of Sec. V-B), FP32."""
    lam = np.asarray(lam, dtype=np.float64)
    return f32(np.minimum(lam - lam.max(), 0.0))


def table3_instance(hours: float, delta: float, *, T: int = 8784, R: int = 200, seed: int = 6):
    """1 MW battery of the given duration on grid step delta, eta = sqrt(0.85) (Sec. V)."""
    S = int(round(hours / delta)) + 1
    lam, prob = iid_prices(T, R, seed=seed)
    eta = float(np.float32(math.sqrt(0.85)))
    return IidInstance(f"iid_T{T}_R{R}_S{S}_d{delta}", T, R, S, float(np.float32(delta)), eta,
                       1.0, lam, prob)


WORKLOADS = {
    "day_hourly_small": day_hourly_small,
    "day_5min": day_5min,
    "year_hourly": year_hourly,
    "day_5min_adjoint": day_5min_adjoint,
}
