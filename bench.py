#!/usr/bin/env python3
"""Throughput of the TWA trajectory hot path on one MI355X.

Workload (the headline configuration): a chain of N = 10^4 atoms, pump
exponent alpha = 1, w = ln(N) Gamma, Gamma = 1, 1024 trajectories, dt = 1e-4,
2e4 stochastic Heun steps of Eq. (S1) with the averaging window over the last
half, the channel-mixing contraction in BF16 on MFMA with FP32 accumulation
and FP32 spin updates.  All inputs are synthetic: the Philox stream of the
method, keyed by seed 0.

One bench "step" is one complete ``twa_run`` of that workload (noise,
contractions, Heun stages, observables); the pump factorisation is built once
before the timed region and reported separately.  ``value`` is
trajectory-atom-steps/s = n_traj * N * n_steps / wall time per run.

The ``roofline`` object refers to the predictor contraction (the larger of the
two contraction launches of a step): algorithmic flops per launch
2 * N * (2N) * (2 n_traj), divided by its mean launch duration from HIP events
recorded by the library on its stream during the timed runs.

``cpu_baseline`` times the FP64 NumPy oracle (test infrastructure) on the
host's cores on a bounded sample of the same workload (a few trajectories for
a few steps at N = 10^4).

``adjoint`` is the second half of the metric: the cost of the pathwise
gradients d<S+S->/d(w, alpha) and dg2/d(w, alpha) (checkpointed forward plus
reverse sweep) relative to a plain forward run of the same configuration
(N = 2000, alpha = 1, w = 2, 2048 trajectories, dt = 1e-4, FP32 contractions,
a checkpoint every 256 steps).  The ratio is per step, so a bounded number of
steps (2048, i.e. 8 checkpoint segments) is timed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trajectory-atom-steps/s at N=1e4 + adjoint d(g2)/d(w,alpha) cost vs forward"
PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3, "fp64": 78.6}
KERNEL_SOURCES = ["paper_2608_10075_amd/csrc/twa_step.hip", "paper_2608_10075_amd/csrc/twa_device.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, precision: str):
    """HBM bytes per launch of the predictor contraction from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stage1_traffic_%s_%s.json" % (workload, precision))
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_sha") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(N, w, alpha, dt, budget_s=15.0, threads=None, pump=None):
    """The FP64 oracle as it stands, timed on a bounded sample of the workload
    (BLAS threads: all, or limited to ``threads``).  ``pump`` = (oracle pump,
    its build time) reuses an oracle pump built earlier (the one-time
    eigendecomposition is not part of the rate); returns (line, pump)."""
    if threads is not None:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=threads):
            return cpu_baseline(N, w, alpha, dt, budget_s, pump=pump)
    from oracle import pump as opump, twa as otwa
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    if pump is None:
        t0 = time.time()
        pump = (opump.build_pump(N, w, alpha), time.time() - t0)
    p, build_s = pump
    B = 4
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=1, seed=0)
    state = otwa.initial_state(0, B, N)
    t0 = time.time()
    state = otwa.run_steps(state, p, cfg, 0, 2)
    per = (time.time() - t0) / 2
    steps = max(2, int(budget_s / max(per, 1e-6)))
    t0 = time.time()
    otwa.run_steps(state, p, cfg, 2, steps)
    el = time.time() - t0
    return {"value": B * N * steps / el, "unit": "trajectory-atom-steps/s", "cores": int(cores),
            "kind": "oracle",
            "sample": "FP64 NumPy oracle, N=%d, %d trajectories x %d Heun steps (%.1f s); pump eigendecomposition "
                      "%.1f s (all cores) not included" % (N, B, steps, el, build_s)}, pump


def adjoint_cost(twa, steps=2048, reps=1):
    """Wall time of twa_adjoint (forward with checkpoints + reverse sweep) for
    dg2/d(w, alpha) divided by the wall time of twa_run on the same
    configuration; also the cost with both objectives (<S+S-> and g2) swept."""
    import torch
    N, B, w, alpha, dt, ck = 2000, 2048, 2.0, 1.0, 1e-4, 256
    pump = twa.build_pump(N, w, alpha)
    twa.run(pump, B, dt, 64, seed=0, precision="fp32")           # warm caches / graphs
    twa.adjoint(pump, B, dt, 256, seed=0, precision="fp32", ckpt_every=ck, objectives=("g2",))
    fwd, adj, adj2 = [], [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.time()
        r = twa.run(pump, B, dt, steps, seed=0, precision="fp32")
        torch.cuda.synchronize()
        t1 = time.time()
        obs, grads = twa.adjoint(pump, B, dt, steps, seed=0, precision="fp32", ckpt_every=ck, objectives=("g2",))
        torch.cuda.synchronize()
        t2 = time.time()
        twa.adjoint(pump, B, dt, steps, seed=0, precision="fp32", ckpt_every=ck)
        torch.cuda.synchronize()
        t3 = time.time()
        fwd.append(t1 - t0)
        adj.append(t2 - t1)
        adj2.append(t3 - t2)
    f, a, a2 = min(fwd), min(adj), min(adj2)
    grads = {k: v for k, v in grads.items() if k.startswith("d_g2")}
    return {"ratio": a / f, "forward_s": f, "adjoint_s": a, "steps": steps, "objective": "g2",
            "ratio_both_objectives": a2 / f,
            "config": {"N": N, "alpha": alpha, "w": w, "n_traj": B, "dt": dt, "precision": "fp32",
                       "ckpt_every": ck, "tile_config": r.obs["tile_config"]},
            "forward_ms_per_step": 1e3 * f / steps, "adjoint_ms_per_step": 1e3 * a / steps,
            "gradients": grads}


def scan_points(n_points=96, seed=0):
    """The uneven phase-diagram scan: N_p = default_rng(0).integers(64, 4097,
    96), (alpha, w) over linspace(0, 3, 12) x logspace(-2, 2, 8) in row-major
    order, seed = point index; dt from the step criterion 0.04 / max(Gamma N,
    lam_max) (below the paper's 0.05) with lam_max bounded by the largest row
    sum of Eq. (2) (the row sums peak at the middle row)."""
    import numpy as np
    Ns = np.random.default_rng(seed).integers(64, 4097, n_points)
    pts = []
    q = 0
    for a in np.linspace(0.0, 3.0, 12):
        for w in np.logspace(-2, 2, 8):
            if q == n_points:
                break
            N = int(Ns[q])
            i = np.arange(N)
            rowmax = float((w / (1.0 + np.abs(i - N // 2)) ** a).sum())
            pts.append((N, float(w), float(a), 0.04 / max(N, rowmax), q))
            q += 1
    return pts


def batch_scan(twa, steps):
    """Batched scan (grouped persistent launches, graph replay, autotuned
    tiles) against the same 96 points run one by one through the plain FP32
    path, and one by one through the Toeplitz path; device time of the step
    loops (pump builds excluded), 512 trajectories, FP32."""
    import torch
    pts = scan_points()
    B = 512
    t0 = time.time()
    res = twa.run_batch(pts, B, steps, precision="fp32")
    torch.cuda.synchronize()
    batch_wall = time.time() - t0
    batch_ms = res[0]["kernel_ms"]
    single_ms = 0.0
    toep_ms = 0.0
    for i, (N, w, a, dt, seed) in enumerate(pts):
        p = twa.build_pump(N, w, a)
        r = twa.run(p, B, dt, steps, seed=seed, point=i, precision="fp32")
        single_ms += r.obs["kernel_ms"]
        p.close()
        lt = twa.build_pump_toeplitz(N, w, a)
        t = twa.run(lt, B, dt, steps, seed=seed, point=i, precision="fp32", pump_path="toeplitz")
        toep_ms += t.obs["kernel_ms"]
    work = sum(B * N * steps for (N, _, _, _, _) in pts)
    crit = [r["step_criterion"] for r in res]
    return {"points": len(pts), "n_traj": B, "steps": steps, "precision": "fp32",
            "N_list": [p[0] for p in pts], "step_criterion_min_max": [min(crit), max(crit)],
            "batched_ms": batch_ms, "single_runs_ms": single_ms, "toeplitz_single_runs_ms": toep_ms,
            "speedup_batched_vs_single": single_ms / batch_ms,
            "speedup_toeplitz_vs_single": single_ms / toep_ms,
            "batched_rate": work / (batch_ms * 1e-3), "unit": "trajectory-atom-steps/s",
            "batch_wall_s_incl_pumps_and_tuning": batch_wall}


def sib_rate(twa, pump, B, dt, prec, steps=400):
    """Device time per step of the semi-implicit midpoint scheme against Heun
    on the headline pump (same three operand sweeps per step)."""
    out = {}
    for integ in ("heun", "sib"):
        twa.run(pump, B, dt, 32, seed=0, precision=prec, integrator=integ)
        r = twa.run(pump, B, dt, steps, seed=0, precision=prec, integrator=integ)
        out[integ + "_ms_per_step"] = r.obs["kernel_ms"] / steps
        out[integ + "_max_norm_dev"] = r.obs["max_norm_dev"]
    out["steps"] = steps
    out["precision"] = prec
    return out


def two_time_cost(twa, N=1000, w=1.0, alpha=1.0, B=4096, dt=1e-4, T=4000, lags=500, prec="fp32"):
    """Cost of the two-time correlation (two tangent-linear response copies
    propagated from the window start, and the lag sums) on the N = 1000,
    4096-trajectory workload: device time of a run with the lag window over
    the last half against the same run without it, and the cost per step
    inside the window relative to a plain step."""
    pump = twa.build_pump(N, w, alpha)
    burn = T // 2
    stride = max(1, (T - burn) // lags)
    twa.run(pump, B, dt, 64, seed=0, precision=prec)
    plain = twa.run(pump, B, dt, T, seed=0, precision=prec, burnin=burn).obs["kernel_ms"]
    twa.run(pump, B, dt, 64, seed=0, precision=prec, burnin=32, n_lags=16, lag_stride=2)
    r = twa.run(pump, B, dt, T, seed=0, precision=prec, burnin=burn, n_lags=lags, lag_stride=stride)
    lagged = r.obs["kernel_ms"]
    per_step = plain / T
    window = (lagged - plain) / (T - burn) + per_step
    return {"config": {"N": N, "w": w, "alpha": alpha, "n_traj": B, "dt": dt, "n_steps": T, "burnin": burn,
                       "n_lags": lags, "lag_stride": stride, "precision": prec},
            "plain_ms": plain, "with_lags_ms": lagged, "plain_ms_per_step": per_step,
            "window_ms_per_step": window, "window_cost_ratio": window / per_step,
            "linewidth": r.obs.get("linewidth")}


def threshold_vs_scan(twa, N=2000, alpha=1.0, B=2048, dt=1e-4, T=2048):
    """Locating a threshold by Newton steps with adjoint gradients against
    forward-only searches, at fixed noise: <S+S->/N = target on a bracket
    found by a coarse scan (target 1, the paper's criterion, when the scan
    crosses it), FP32, tolerance 1e-6 relative in w."""
    import numpy as np
    import torch
    burn = T // 2
    grid = np.geomspace(0.5, 64.0, 8)
    vals, t_fwd = [], []
    for w in grid:
        p = twa.build_pump(N, float(w), alpha)
        torch.cuda.synchronize()
        t0 = time.time()
        r = twa.run(p, B, dt, T, seed=0, precision="fp32", burnin=burn)
        torch.cuda.synchronize()
        t_fwd.append(time.time() - t0)
        vals.append(r.obs["SpSm"] / N)
        p.close()
    vals = np.array(vals)
    cross = [i for i in range(len(grid) - 1) if (vals[i] - 1.0) * (vals[i + 1] - 1.0) < 0]
    if cross:
        i, target = cross[0], 1.0
    else:
        i = int(np.argmax(np.abs(np.diff(vals))))
        target = 0.5 * (vals[i] + vals[i + 1])
    lo, hi = float(grid[i]), float(grid[i + 1])
    tol = 1e-6 * hi
    torch.cuda.synchronize()
    t0 = time.time()
    w_root, f_root, it = twa.find_threshold(N, alpha, B, dt, T, 0, objective="spsm_n", target=target, w_lo=lo,
                                            w_hi=hi, tol_w=tol, precision="fp32", burnin=burn)
    torch.cuda.synchronize()
    newton_s = time.time() - t0
    fwd = float(np.median(t_fwd))
    n_bisect = int(math.ceil(math.log2((hi - lo) / tol)))
    return {"config": {"N": N, "alpha": alpha, "n_traj": B, "dt": dt, "n_steps": T, "precision": "fp32"},
            "objective": "spsm_n", "target": target, "bracket": [lo, hi], "w_root": w_root, "residual": f_root,
            "gradient_evaluations": it, "newton_s": newton_s, "forward_run_s": fwd,
            "bisection_forward_runs_same_tol": n_bisect,
            "speedup_vs_bisection": n_bisect * fwd / newton_s,
            "uniform_scan_points_same_time": int(newton_s / fwd),
            "uniform_scan_resolution_same_time": (hi - lo) / max(1, int(newton_s / fwd))}


def toeplitz_rate(twa, N, w, alpha, B, dt, T, dense_value):
    """The same workload through the circulant embedding of Eq. (2) (FFT
    drift and circulant pump noise, equal in law to the dense path), FP32,
    one full run after a short warm-up run."""
    import torch
    light = twa.build_pump_toeplitz(N, w, alpha)
    twa.run(light, B, dt, 256, seed=0, precision="fp32", pump_path="toeplitz")
    torch.cuda.synchronize()
    t0 = time.time()
    r = twa.run(light, B, dt, T, seed=0, precision="fp32", pump_path="toeplitz")
    torch.cuda.synchronize()
    wall = time.time() - t0
    value = B * N * T / wall
    M = 256
    while M < 2 * N - 2:
        M *= 2
    return {"value": value, "unit": "trajectory-atom-steps/s", "precision": "fp32", "wall_s": wall,
            "kernel_ms": r.obs["kernel_ms"], "speedup_vs_dense": value / dense_value, "embedding_size": M,
            "observables": {k: r.obs[k] for k in ("Sz", "SpSm", "g2", "Sz_se", "SpSm_se", "g2_se")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--tile-config", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-toeplitz", action="store_true")
    ap.add_argument("--sib", action="store_true", help="also time the semi-implicit scheme against Heun")
    ap.add_argument("--threshold", action="store_true",
                    help="also time a Newton threshold search against forward-only searches")
    ap.add_argument("--two-time", action="store_true",
                    help="also time the two-time correlation window (N = 1000, 4096 trajectories, FP32)")
    ap.add_argument("--batch-scan", type=int, default=0,
                    help="also time the 96-point scan for this many steps (batched vs single runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (trajectories would shard "
              "across GPUs with one all-reduce of the accumulators at the end)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    import paper_2608_10075_amd as twa

    N, alpha, B, dt, T = 10000, 1.0, 1024, 1e-4, 20000
    w = math.log(N)
    prec = args.precision
    workload = "n1e4"
    print("[bench] building pump N=%d alpha=%g w=%.4f" % (N, alpha, w), file=sys.stderr, flush=True)
    t0 = time.time()
    pump = twa.build_pump(N, w, alpha)
    torch.cuda.synchronize()
    pump_s = time.time() - t0

    def one(timing):
        return twa.run(pump, B, dt, T, seed=0, precision=prec, tile_config=args.tile_config, timing=timing)

    for i in range(args.warmup):
        print("[bench] warmup run %d/%d" % (i + 1, args.warmup), file=sys.stderr, flush=True)
        one(True)
    torch.cuda.synchronize()
    t0 = time.time()
    results = []
    for i in range(args.steps):
        print("[bench] timed run %d/%d" % (i + 1, args.steps), file=sys.stderr, flush=True)
        results.append(one(True))
    torch.cuda.synchronize()
    wall = time.time() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = B * N * T * args.steps / wall

    s1_ms = sum(r.obs["stage1_ms"] for r in results)
    s1_n = sum(r.obs["stage1_launches"] for r in results)
    s2_ms = sum(r.obs["stage2_ms"] for r in results)
    s2_n = sum(r.obs["stage2_launches"] for r in results)
    flops1 = 2.0 * N * (2 * N) * (2 * B)
    flops2 = 2.0 * N * N * (2 * B)
    ach1 = flops1 / (s1_ms / s1_n * 1e-3) / 1e12
    ach2 = flops2 / (s2_ms / s2_n * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    obs = results[-1].obs
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": "TWA chain N=10000 alpha=1 w=ln(N) Gamma=1, 1024 trajectories, dt=1e-4, %d Heun "
                               "steps, window = last half, %s channel-mixing contraction" % (T, prec),
                   "N": N, "alpha": alpha, "w": w, "n_traj": B, "dt": dt, "n_steps": T, "precision": prec,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": ach1, "peak": peak, "unit": "TFLOP/s", "frac": ach1 / peak,
                     "traffic": traffic_from_profiles(workload, prec),
                     "kernel": "heun_stage_kernel stage 1 (predictor contraction, K = 2N)",
                     "flops_per_launch": flops1, "mean_launch_ms": s1_ms / s1_n},
        "roofline_stage2": {"achieved": ach2, "peak": peak, "unit": "TFLOP/s", "frac": ach2 / peak,
                            "mean_launch_ms": s2_ms / s2_n, "flops_per_launch": flops2},
        "pump_build_s": pump_s,
        "observables": {k: obs[k] for k in ("Sz", "SpSm", "g2", "Sz_se", "SpSm_se", "g2_se", "max_norm_dev",
                                             "step_criterion")},
        "tile_config": obs["tile_config"],
    }
    if not args.no_toeplitz:
        print("[bench] Toeplitz fast path on the same workload (FP32)", file=sys.stderr, flush=True)
        line["toeplitz_path"] = toeplitz_rate(twa, N, w, alpha, B, dt, T, value)
    if args.sib:
        print("[bench] semi-implicit scheme vs Heun", file=sys.stderr, flush=True)
        line["sib_vs_heun"] = sib_rate(twa, pump, B, dt, prec)
    if args.threshold:
        print("[bench] threshold search (N=2000, FP32)", file=sys.stderr, flush=True)
        line["threshold"] = threshold_vs_scan(twa)
    if args.two_time:
        print("[bench] two-time correlation window (N=1000, FP32)", file=sys.stderr, flush=True)
        line["two_time"] = two_time_cost(twa)
    if args.batch_scan > 0:
        print("[bench] batched scan, 96 points, %d steps" % args.batch_scan, file=sys.stderr, flush=True)
        line["batch_scan"] = batch_scan(twa, args.batch_scan)
    if not args.no_adjoint:
        print("[bench] adjoint cost ratio (N=2000, FP32)", file=sys.stderr, flush=True)
        line["adjoint"] = adjoint_cost(twa)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"], opump_ = cpu_baseline(N, w, alpha, dt)
        line["cpu_baseline_single_core"], _ = cpu_baseline(N, w, alpha, dt, budget_s=8.0, threads=1, pump=opump_)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
