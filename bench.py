#!/usr/bin/env python
"""Throughput of the GPU backward induction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload year_hourly]

The default workload is the year-long hourly solve (T = 8760 stages, K = 50 price states,
S = 2001 SoC points, moves of +-500 steps, a 5 $ start cost): the largest single solve.
A step is one full backward induction of the workload: for every stage the expectation
W_t = P_t V_{t+1} (MFMA) and the max-plus Bellman sweep with argmax, writing V_1 and all
int16 policies to HBM.  The metric is feasible state-action updates per second (the
(t, k, s, j) candidates of the solve over the wall time of a step), inputs resident in
HBM before the timed region.  One JSON line is printed; besides the required fields it
carries:
  roofline      the Bellman-sweep kernel (dominant): feasible candidates per launch over
                its average launch time, measured with HIP events on the solve's stream
                in a second pass of the same steps right after the timed ones, against
                the FP32 vector bound (an add and a max per candidate at 32 lanes per
                clock per SIMD);
  cpu_baseline  the FP64 oracle timed on this host's cores on a bounded sample of the
                same workload (its last stages);
  extra         the five-minute day solve, the adjoint/value time ratio and the
                batched/looped comparison, each on the same GPU, the paper-mode Table 3
                shapes, and CPU timings of the oracle and of Algorithm 1 in NumPy on the
                smaller workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

# Peak of the sweep: the FP32 vector rate, 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 7.86e13
# lane-operations/s (the published 157.3 TFLOP/s counts an FMA as two), with one candidate
# costing one add and one max (two operations; two-input add and fma issue at 2 clocks per
# wave64 instruction, v_max3_f32 at 4, so a pair of candidates costs 2 adds + 1 max3 = 8
# clocks either way): 3.93e13 candidates/s.
VALU_LANE_OPS = 256 * 4 * 32 * 2.4e9
SWEEP_PEAK_GUPD = VALU_LANE_OPS / 2.0 / 1e9
# Dense FP32 matrix-core peak of the MI355X (published): 157.3 TFLOP/s.
MFMA_F32_PEAK_TFLOPS = 157.3


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


class ClockSampler:
    """The GPU's current graphics clock level (MHz), read from the driver's
    pp_dpm_sclk table (the line marked '*') of the card at the device's PCI address,
    every few ms on a thread while a `with` block runs."""

    def __init__(self, torch, period_s=0.004):
        self.period, self.samples, self.path = period_s, [], None
        self._stop = threading.Event()
        try:
            pr = torch.cuda.get_device_properties(0)
            bdf = f"{pr.pci_domain_id:04x}:{pr.pci_bus_id:02x}:{pr.pci_device_id:02x}.0"
            for card in sorted(os.listdir("/sys/class/drm")):
                dev = os.path.join("/sys/class/drm", card, "device")
                f = os.path.join(dev, "pp_dpm_sclk")
                if card.startswith("card") and os.path.exists(f) and \
                        os.path.basename(os.path.realpath(dev)) == bdf:
                    self.path = f
                    break
        except Exception:
            self.path = None

    def _read(self):
        with open(self.path) as fh:
            for line in fh:
                if line.rstrip().endswith("*"):
                    return float(line.split(":")[1].strip().lower().split("mhz")[0])
        return None

    def _run(self):
        while not self._stop.is_set():
            try:
                v = self._read()
            except Exception:
                return
            if v is not None:
                self.samples.append(v)
            self._stop.wait(self.period)

    def __enter__(self):
        self._t = None
        if self.path:
            self._t = threading.Thread(target=self._run, daemon=True)
            self._t.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self._t is not None:
            self._t.join()

    def summary(self):
        if not self.samples:
            return None
        v = sorted(self.samples)
        return {"median": v[len(v) // 2], "min": v[0], "max": v[-1], "samples": len(v),
                "source": "driver pp_dpm_sclk current level during the event-timed solves"}


def timed_solves(dp, torch, inst, steps, warmup, clock=None):
    """Wall time per step over `steps` solves (no instrumentation), then identical solves
    with HIP event pairs (created without the system-scope fence) on the solve's stream
    around every sweep and expectation launch, as many solves as keep the event count
    within about 20k (at least one); event packets between launches slow the steps down, so they are kept
    out of the timed steps.  The clock sampler, if given, runs during the event-timed
    solves only."""
    lam = torch.from_numpy(inst.lam).cuda()
    P = torch.from_numpy(inst.P).cuda()
    solver = dp.Solver(lam, P, inst.storage, store_all=False, policy=True)
    for _ in range(warmup):
        solver.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dp.lib().dp_set_timing(2)
    import contextlib
    with clock if clock is not None else contextlib.nullcontext():
        for _ in range(max(1, min(steps, 10000 // inst.T))):
            solver.run()
        torch.cuda.synchronize()
    timing = dp.kernel_timing()
    dp.kernel_timing(False)
    del solver
    return (t1 - t0) / steps, timing


HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "paper_2511_15629_amd", "csrc", "dp_kernels.hip")


def traffic_file(workload: str) -> str:
    return os.path.join(HERE, "profiles", f"sweep_traffic_{workload}.txt")


def measured_traffic(workload: str):
    """HBM bytes per sweep launch from the committed counter summary of this workload (two
    rocprofv3 --pmc passes, calibrated on a copy of known size), or None when there is
    none or the kernel source has changed since the counters were taken."""
    import hashlib
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if not line.startswith("#") and ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != digest:
        return None
    return int(fields["bytes_per_launch"])


def roofline_of(inst, timing, traffic=None):
    sweep_ms, n_sweep, exp_ms, n_exp = timing
    per_launch = inst.candidates() / inst.T            # candidates per sweep launch (avg)
    avg_s = sweep_ms / 1e3 / max(n_sweep, 1)
    achieved = per_launch / avg_s / 1e9
    if n_exp == 0:
        # one launch per stage: the expectation is formed inside the sweep launch
        return {
            "bound": "alu", "achieved": round(achieved, 1), "peak": round(SWEEP_PEAK_GUPD, 1),
            "unit": "Gupd/s", "frac": round(achieved / SWEEP_PEAK_GUPD, 4), "traffic": traffic,
            "traffic_GBps": None if traffic is None else round(traffic / avg_s / 1e9, 1),
            "kernel": "sweep_kernel (expectation fused)", "avg_launch_us": round(avg_s * 1e6, 3),
            "launches": n_sweep,
            # the work unit is the feasible candidate (one VALU lane-instruction each in a
            # direct evaluation); the kernel takes window maxima by prefix/suffix scans, so
            # its time is set by staging the expectation row and by per-stage latency
            "work": "feasible candidates per launch at 1 VALU lane-op each",
        }
    exp_avg = max(exp_ms / 1e3 / max(n_exp, 1), 1e-12)
    exp_flop = 2.0 * inst.K * inst.K * inst.storage.S
    return {
        "bound": "alu", "achieved": round(achieved, 1), "peak": round(SWEEP_PEAK_GUPD, 1),
        "unit": "Gupd/s", "frac": round(achieved / SWEEP_PEAK_GUPD, 4), "traffic": traffic,
        "traffic_GBps": None if traffic is None else round(traffic / avg_s / 1e9, 1),
        "kernel": "sweep_kernel", "avg_launch_us": round(avg_s * 1e6, 3),
        "launches": n_sweep,
        "expectation_avg_launch_us": round(exp_avg * 1e6, 3),
        # the expectation W_t = P_t V_{t+1} on the FP32 matrix cores: 2 K^2 S flop per launch
        "expectation": {"bound": "mfma", "achieved": round(exp_flop / exp_avg / 1e12, 3),
                        "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(exp_flop / exp_avg / 1e12 / MFMA_F32_PEAK_TFLOPS, 4),
                        "kernel": "contract_packed_kernel"},
    }


def cpu_baseline(inst, budget_s=15.0):
    """The FP64 oracle as it stands, on every host core, over the last n stages of the
    workload (n chosen from a short probe so that the run takes about budget_s), and on
    one thread over its last few stages.  Rates are feasible candidates per second; every
    stage of a workload has the same candidate count."""
    import oracle
    cores = host_cores()
    per_stage = inst.candidates() / inst.T

    def run(n, threads):
        t0 = time.perf_counter()
        oracle.solve(inst.storage, inst.lam[-n:], inst.P[-n:], keep_all=False,
                     want_policy=True, threads=threads)
        return time.perf_counter() - t0

    n0 = min(inst.T, 4)
    dt0 = run(n0, cores)
    n = int(max(n0, min(inst.T, budget_s / max(dt0 / n0, 1e-9))))
    dt = run(n, cores)
    n1 = min(inst.T, 4 if per_stage > 2e7 else 24)
    dt1 = run(n1, 1)
    return {"value": round(per_stage * n / dt, 1), "unit": "updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"the last {n} of {inst.T} stages of {inst.name} ({dt:.1f} s; FP64 C "
                      f"loops, OpenMP over price states, {cores} threads)",
            "single_thread": {"value": round(per_stage * n1 / dt1, 1),
                              "sample": f"the last {n1} stages of {inst.name}, 1 thread"}}


def cpu_timings():
    """CPU times of the other workloads: the oracle (FP64 C loops, all cores) on the hourly
    day, the five-minute day and the adjoint of the five-minute day (the oracle's adjoint
    under the oracle's own policies, after its solve), and Algorithm 1 as the paper runs it
    (NumPy, materialised S x P x R payoff tensor, one price sample per price state) on the
    hourly day (whole) and on the five-minute day shapes (a few stages)."""
    import numpy as np
    import oracle
    from oracle import alg1
    import workloads as wl
    cores = host_cores()
    out = {"cores": cores}
    for inst in (wl.day_hourly_small(), wl.day_5min()):
        t0 = time.perf_counter()
        ref = oracle.solve(inst.storage, inst.lam, inst.P, keep_all=True, threads=cores)
        dt = time.perf_counter() - t0
        out[f"oracle_{inst.name}"] = {"s": round(dt, 3),
                                      "updates_per_s": round(inst.candidates() / dt, 1)}
        if inst.K == 100:
            seed = wl.default_seed(inst.K, inst.storage.S).astype(np.float64)
            t0 = time.perf_counter()
            oracle.adjoint(inst.storage, inst.lam, inst.P, ref["V"], ref["policy"], seed,
                           threads=cores)
            da = time.perf_counter() - t0
            out[f"oracle_adjoint_{inst.name}"] = {"s": round(da, 3),
                                                  "adjoint_over_solve": round(da / dt, 3)}
        del ref
        # Algorithm 1 in NumPy on the same shapes: the integer-step action grid of the
        # window, R = K price samples (the stage's levels) with equal probabilities
        st = inst.storage
        s_hat = np.arange(st.S) * float(st.delta)
        p_hat = np.array([-(k * float(st.delta) / float(st.eta_c)) for k in range(st.w_up, 0, -1)]
                         + [0.0] + [k * float(st.delta) * float(st.eta_d)
                                    for k in range(1, st.w_down + 1)])
        nT = inst.T if inst.K <= 10 else 3
        pi = np.full(inst.K, 1.0 / inst.K)
        pre = alg1.precompute(s_hat, p_hat, float(st.eta_c))
        V = np.zeros(st.S)
        t0 = time.perf_counter()
        for t in range(inst.T, inst.T - nT, -1):
            V, _ = alg1.stage(pre, p_hat, inst.lam[t - 1], pi, V)
        dt = time.perf_counter() - t0
        out[f"algorithm1_numpy_{inst.name}"] = {
            "stages": nT, "s": round(dt, 3),
            "sample_action_pairs_per_s": round(st.S * p_hat.size * inst.K * nT / dt, 1),
            "threads": "NumPy (single-threaded element-wise ops)"}
    return out


def adjoint_ratio(dp, torch, inst, reps=5):
    lam = torch.from_numpy(inst.lam).cuda()
    P = torch.from_numpy(inst.P).cuda()
    seed = torch.zeros(inst.K, inst.storage.S, device="cuda")
    seed[:, 0] = 1.0 / inst.K
    res = {}
    for every in (0, 16):
        def value_only():
            if every:
                return dp.solve(lam, P, inst.storage, store_all=False, policy=False, ckpt_every=every)
            return dp.solve(lam, P, inst.storage, store_all=True, policy=True)

        def value_and_adjoint():
            out = value_only()
            if every:
                dp.adjoint(lam, P, inst.storage, seed, ckpt=out["ckpt"], ckpt_every=every)
            else:
                dp.adjoint(lam, P, inst.storage, seed, V_all=out["V"], policy=out["policy"])

        for f in (value_only, value_and_adjoint):
            f()
        torch.cuda.synchronize()
        tv = []
        for f in (value_only, value_and_adjoint):
            t0 = time.perf_counter()
            for _ in range(reps):
                f()
            torch.cuda.synchronize()
            tv.append((time.perf_counter() - t0) / reps)
        res["ckpt16" if every else "full_storage"] = {
            "value_ms": round(tv[0] * 1e3, 3), "value_adjoint_ms": round(tv[1] * 1e3, 3),
            "ratio": round(tv[1] / tv[0], 3)}
    return res


def batch_compare(dp, torch, reps=2):
    import workloads as wl
    insts = wl.fleet_5min()
    import tempfile
    cache_path = os.path.join(tempfile.gettempdir(), "dpgpu_tune_cache.txt")
    t0 = time.perf_counter()
    plan = dp.BatchPlan([(i.T, i.K, i.storage) for i in insts], tune_cache=cache_path)
    plan_s = time.perf_counter() - t0
    cache = {}
    lams, Ps, V1s, pols = [], [], [], []
    for i in insts:
        lams.append(torch.from_numpy(i.lam).cuda())
        key = id(i.P)
        if key not in cache:
            cache[key] = torch.from_numpy(i.P).cuda()
        Ps.append(cache[key])
        V1s.append(torch.empty(i.K, i.storage.S, device="cuda"))
        pols.append(torch.empty(i.T, i.K, i.storage.S, dtype=torch.int16, device="cuda"))
    cand = sum(i.candidates() for i in insts)
    out = {"instances": len(insts), "candidates": cand, "plan_create_s": round(plan_s, 2),
           "plan": plan.describe().strip().splitlines()}
    for name, kw in (("batched", {}), ("batched_no_graph", dict(graph=False)),
                     ("looped", dict(looped=True))):
        plan.solve(lams, Ps, V1s, pols, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.solve(lams, Ps, V1s, pols, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"ms": round(dt * 1e3, 2), "Gupd_per_s": round(cand / dt / 1e9, 1),
                     # whole solve (sweeps and expectations) against the sweep's VALU peak
                     "frac_of_valu_peak": round(cand / dt / 1e9 / SWEEP_PEAK_GUPD, 4)}
    out["speedup"] = round(out["looped"]["ms"] / out["batched"]["ms"], 3)
    plan.close()
    return out


# Full-year solve times of the stagewise-independent variant on the power grid as the paper
# reports them (Table 3: 8784 hourly stages, 200 samples; NumPy on a 32-core Xeon, CuPy on an
# L40S).  Context for the same workload shapes here, not a target of the headline metric.
TABLE3_PAPER_S = {(4, 0.1): (3.98, 2.77), (20, 0.1): (18.29, 2.81), (100, 0.1): (98.12, 2.94),
                  (4, 0.01): (397.80, 4.88), (20, 0.01): (1996.02, 19.17),
                  (100, 0.01): (9972.64, 86.67)}


def table3_independent(dp, torch):
    """One full-year value solve per Table 3 row (V_0 only, as Algorithm 1 returns)."""
    import workloads as wl
    rows = []
    for hours, delta in wl.TABLE3:
        inst = wl.table3_instance(hours, delta)
        lam = torch.from_numpy(inst.lam).cuda()
        prob = torch.from_numpy(inst.prob).cuda()
        P = dp.power_grid_size(inst.S, inst.delta, inst.eta, inst.p_bar)[0]
        dp.solve_independent(lam[:8], prob[:8], inst.S, inst.delta, inst.eta, inst.p_bar)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dp.solve_independent(lam, prob, inst.S, inst.delta, inst.eta, inst.p_bar)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cpu_s, gpu_s = TABLE3_PAPER_S[(hours, delta)]
        rows.append({"hours": hours, "S": inst.S, "P": P, "T": inst.T, "R": inst.R,
                     "s": round(dt, 4),
                     "sample_action_pairs_per_s": round(inst.S * P * inst.R * inst.T / dt, 1),
                     "frac_of_valu_peak": round(inst.S * P * inst.R * inst.T / dt / 1e9
                                                / SWEEP_PEAK_GUPD, 4),
                     "paper_gpu_s": gpu_s, "paper_cpu_s": cpu_s,
                     "paper_gpu_over_this": round(gpu_s / dt, 1)})
        del lam, prob
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="year_hourly")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--extra", default="day,adjoint,batch,table3,cpu",
                    help="comma-separated extras to run after the headline line's steps")
    ap.add_argument("--stages", type=int, default=0,
                    help="profiling aid: solve only the workload's first N stages (counter runs "
                         "serialise every launch); the JSON line then names the truncated workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the steps, copy 256 MiB device-to-device once (a kernel of known "
                         "traffic for calibrating hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on a single GPU (asked for {args.gpus}); batches "
              "shard across GPUs by instance, which this benchmark does not run",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl
    import paper_2511_15629_amd as dp

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    inst = wl.WORKLOADS[args.workload]()
    if 0 < args.stages < inst.T:
        import dataclasses
        inst = dataclasses.replace(inst, name=f"{inst.name}_first{args.stages}", T=args.stages,
                                   lam=inst.lam[:args.stages], P=inst.P[:args.stages])
    clock = ClockSampler(torch)
    sec, timing = timed_solves(dp, torch, inst, args.steps, args.warmup, clock)
    cand = inst.candidates()
    st = inst.storage
    dense = inst.T * inst.K * st.S * (st.w_up + st.w_down + 1)
    line = {
        "metric": "DP state-action updates/s", "value": round(cand / sec, 1), "unit": "updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": inst.name, "T": inst.T, "K": inst.K, "S": st.S,
                   "w_up": st.w_up, "w_down": st.w_down, "candidates_per_step": cand,
                   "outputs": "V_1 f32 + all int16 policies", "parallelism": "single GPU"},
        "roofline": roofline_of(inst, timing, measured_traffic(args.workload)),
        "dense_equivalent": {"updates_per_step": dense, "updates_per_s": round(dense / sec, 1),
                             "note": "T K S (W_c + W_d + 1): the full window at every level, "
                                     "as a dense action grid counts it"},
        "sclk_mhz": clock.summary(),
    }
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(inst)
    wanted = set() if args.no_extra else {x for x in args.extra.split(",") if x}
    if wanted:
        extra = {}
        for key, make in (("day", wl.day_5min), ("year", wl.year_hourly)):
            if key in wanted and make.__name__ != args.workload:
                other = make()
                osec, otim = timed_solves(dp, torch, other, 5 if other.T < 1000 else 2, 1)
                extra[make.__name__] = {"workload": other.name, "ms": round(osec * 1e3, 3),
                                        "updates_per_s": round(other.candidates() / osec, 1),
                                        "roofline": roofline_of(other, otim,
                                                                measured_traffic(make.__name__))}
                del other
        if "adjoint" in wanted:
            extra["adjoint_vs_value"] = adjoint_ratio(dp, torch, wl.day_5min_adjoint())
        if "batch" in wanted:
            extra["batched_vs_looped"] = batch_compare(dp, torch)
        if "table3" in wanted:
            extra["table3_independent"] = table3_independent(dp, torch)
        if "cpu" in wanted:
            extra["cpu_timings"] = cpu_timings()
        line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
