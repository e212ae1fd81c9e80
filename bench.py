#!/usr/bin/env python3
"""Throughput of the TWA trajectory hot path on one MI355X.

Workload (the headline configuration): a chain of N = 10^4 atoms, pump
exponent alpha = 1, w = ln(N) Gamma, Gamma = 1, 1024 trajectories, dt = 1e-4,
the channel-mixing contraction in BF16 on MFMA with FP32 accumulation and FP32
spin updates, integrated with the spin-length-preserving semi-implicit scheme
the paper uses (the stochastic Heun scheme drifts |s|^2 by 0.47 at this step
size and is reported beside it).  All inputs are synthetic: the Philox stream
of the method, keyed by seed 0.

One bench "step" is 1000 integration steps of the whole hot path (noise,
contractions, stage updates, collective sums, window observables) over the
1024-trajectory batch.  ``--steps K`` times ONE ``twa_run`` of K * 1000
integration steps (averaging window over its last half), so ``--steps 20``
times exactly the 2e4-step headline run; ``--warmup W`` runs W * 1000
untimed integration steps first.  The pump factorisation is built once
before the timed region and reported separately.  ``value`` is
trajectory-atom-steps/s = n_traj * N * (K * 1000) / wall.

The ``roofline`` object refers to the predictor contraction (the larger of the
two contraction launches of a step): algorithmic flops per launch
2 * N * (2N) * (2 n_traj), divided by its mean launch duration from HIP events
recorded by the library on its stream during the timed run.

Beside the headline (each skippable):
  * ``heun``: the same run with the stochastic Heun integrator and the shift
    of its observables against the semi-implicit run, in standard errors;
  * ``precision``: the headline workload for 2000 steps in FP64, FP32, split
    BF16 (hi + lo), BF16 and FP16: time per step, speed-up over FP32 and the
    error of <S^z>, <S+S-> and g2 against FP64 (same noise);
  * ``linewidth_precision``: the linewidth of the two-time correlation on the
    N = 1000 workload in FP64, FP32, split BF16, BF16 and FP16;
  * ``toeplitz_path``: the headline workload through the circulant embedding
    of Eq. (2), FP32;
  * ``adjoint``: the second half of the metric, wall(twa_adjoint for
    dg2/d(w, alpha)) / wall(twa_run) at N = 2000, 2048 trajectories, FP32;
  * ``cpu_baseline``: the FP64 NumPy oracle (test infrastructure) on the host's
    cores on a bounded sample of the headline workload (32 trajectories).

Profiling modes: ``--copy-calibration`` (one 1 GiB device copy, the scale of
the FETCH_SIZE / WRITE_SIZE counters), ``--toeplitz-only`` (the Toeplitz
kernel on the headline workload, 256 + 512 steps).
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
PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}
KERNEL_SOURCES = ["paper_2608_10075_amd/csrc/twa_step_impl.h", "paper_2608_10075_amd/csrc/twa_device.h"]
STEPS_PER_BENCH_STEP = 1000


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, precision: str, integrator: str):
    """HBM bytes per launch of the predictor contraction from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stage1_traffic_%s_%s_%s.json" % (workload, precision, integrator))
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_sha") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(N, w, alpha, dt, integrator, budget_s=15.0, threads=None, pump=None, B=32):
    """The FP64 oracle as it stands, timed on a bounded sample of the workload
    (B trajectories, BLAS threads: all, or limited to ``threads``).  ``pump`` =
    (oracle pump, its build time) reuses an oracle pump built earlier (the
    one-time eigendecomposition is not part of the rate); returns (line, pump)."""
    if threads is not None:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=threads):
            return cpu_baseline(N, w, alpha, dt, integrator, budget_s, pump=pump, B=B)
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
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=1, seed=0, integrator=integrator)
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
            "sample": "FP64 NumPy oracle (%s integrator), N=%d, %d trajectories x %d steps (%.1f s); pump "
                      "eigendecomposition %.1f s not included" % (integrator, N, B, steps, el, build_s)}, pump


def adjoint_cost(twa, steps=2048, reps=1):
    """Wall time of twa_adjoint (forward with checkpoints + reverse sweep) for
    dg2/d(w, alpha) divided by the wall time of twa_run on the same
    configuration; also the cost with both objectives (<S+S-> and g2) swept.
    Heun (the adjoint's integrator) at dt = 1e-4 (step criterion 0.2) drifts
    the spin lengths past the default check, so the check is off here and the
    drift is reported."""
    import torch
    N, B, w, alpha, dt, ck = 2000, 2048, 2.0, 1.0, 1e-4, 256
    pump = twa.build_pump(N, w, alpha)
    twa.run(pump, B, dt, 64, seed=0, precision="fp32", norm_tol=-1)           # warm caches / graphs
    twa.adjoint(pump, B, dt, 256, seed=0, precision="fp32", ckpt_every=ck, objectives=("g2",), norm_tol=-1)
    fwd, adj, adj2 = [], [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.time()
        r = twa.run(pump, B, dt, steps, seed=0, precision="fp32", norm_tol=-1)
        torch.cuda.synchronize()
        t1 = time.time()
        print("[bench]   forward %d steps: %.1f s" % (steps, t1 - t0), file=sys.stderr, flush=True)
        obs, grads = twa.adjoint(pump, B, dt, steps, seed=0, precision="fp32", ckpt_every=ck, objectives=("g2",),
                                 norm_tol=-1)
        torch.cuda.synchronize()
        t2 = time.time()
        print("[bench]   adjoint for g2: %.1f s" % (t2 - t1), file=sys.stderr, flush=True)
        twa.adjoint(pump, B, dt, steps, seed=0, precision="fp32", ckpt_every=ck, norm_tol=-1)
        torch.cuda.synchronize()
        t3 = time.time()
        print("[bench]   adjoint for both objectives: %.1f s" % (t3 - t2), file=sys.stderr, flush=True)
        fwd.append(t1 - t0)
        adj.append(t2 - t1)
        adj2.append(t3 - t2)
    f, a, a2 = min(fwd), min(adj), min(adj2)
    # the same reverse sweep in split BF16 (FP32-class operands), against the
    # FP32 forward run and the FP32 gradients
    twa.adjoint(pump, B, dt, 256, seed=0, precision="bf16x3", ckpt_every=ck, objectives=("g2",), norm_tol=-1)
    torch.cuda.synchronize()
    t4 = time.time()
    _, g3 = twa.adjoint(pump, B, dt, steps, seed=0, precision="bf16x3", ckpt_every=ck, objectives=("g2",),
                        norm_tol=-1)
    torch.cuda.synchronize()
    a3 = time.time() - t4
    print("[bench]   adjoint for g2 in split BF16: %.1f s" % a3, file=sys.stderr, flush=True)
    split = {"adjoint_s": a3, "ratio_vs_fp32_forward": a3 / f, "speedup_vs_fp32_adjoint": a / a3,
             "gradients": {k: v for k, v in g3.items() if k.startswith("d_g2")},
             "rel_diff_vs_fp32": {k: abs(g3[k] - grads[k]) / abs(grads[k]) for k in ("d_g2_dw", "d_g2_dalpha")}}
    grads = {k: v for k, v in grads.items() if k.startswith("d_g2")}
    return {"ratio": a / f, "forward_s": f, "adjoint_s": a, "steps": steps, "objective": "g2",
            "ratio_both_objectives": a2 / f,
            "config": {"N": N, "alpha": alpha, "w": w, "n_traj": B, "dt": dt, "precision": "fp32",
                       "ckpt_every": ck, "tile_config": r.obs["tile_config"], "integrator": "heun"},
            "forward_ms_per_step": 1e3 * f / steps, "adjoint_ms_per_step": 1e3 * a / steps,
            "max_norm_dev": obs["max_norm_dev"], "gradients": grads, "split_bf16": split}


def gradient_check(twa, steps, prec, hs):
    """dg2/dw on the adjoint workload's path (N = 2000, 2048 trajectories,
    fixed noise) by the forward-mode tangent and by central differences of
    the forward run at w +- h (pumps rebuilt), for each h."""
    N, B, w, alpha, dt = 2000, 2048, 2.0, 1.0, 1e-4
    pump = twa.build_pump(N, w, alpha)
    _, tg = twa.tangent_w(pump, B, dt, steps, seed=0, precision=prec, norm_tol=-1)
    print("[bench]   forward-mode dg2/dw: %.6g" % tg["d_g2_dw"], file=sys.stderr, flush=True)
    fd = {}
    for h in hs:
        g2 = []
        for sgn in (1, -1):
            ph = twa.build_pump(N, w + sgn * h, alpha)
            g2.append(twa.run(ph, B, dt, steps, seed=0, precision=prec, norm_tol=-1).obs["g2"])
            ph.close()
        fd["%g" % h] = (g2[0] - g2[1]) / (2 * h)
        print("[bench]   central difference (h = %g): %.6g" % (h, fd["%g" % h]), file=sys.stderr, flush=True)
    return {"steps": steps, "precision": prec, "d_g2_dw_forward_mode": tg["d_g2_dw"],
            "d_g2_dw_central_difference_by_h": fd}


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


def batch_singles(twa, steps, integrator="sib", precision="fp32"):
    """The 96 points of the scan one by one through the plain FP32 path only
    (the single-run side of the batched comparison, for step counts where
    both sides do not fit one run); device time of the step loops."""
    pts = scan_points()
    B = 512
    single_ms = 0.0
    for i, (N, w, a, dt, seed) in enumerate(pts):
        p = twa.build_pump(N, w, a)
        r = twa.run(p, B, dt, steps, seed=seed, point=i, precision=precision, integrator=integrator)
        single_ms += r.obs["kernel_ms"]
        p.close()
        print("[bench]   single run %d/%d (N = %d): %.1f ms" % (i + 1, len(pts), N, r.obs["kernel_ms"]),
              file=sys.stderr, flush=True)
    work = sum(B * N * steps for (N, _, _, _, _) in pts)
    flops = sum(12.0 * N * N * B * steps for (N, _, _, _, _) in pts)
    return {"points": len(pts), "n_traj": B, "steps": steps, "precision": precision, "integrator": integrator,
            "single_runs_ms": single_ms, "single_rate": work / (single_ms * 1e-3), "unit": "trajectory-atom-steps/s",
            "single_tflops": flops / (single_ms * 1e-3) / 1e12}


def batch_scan(twa, steps, integrator="sib", singles=True, precision="fp32"):
    """Batched scan (grouped persistent launches, graph replay, autotuned
    tiles) against the same 96 points run one by one through the plain FP32
    path, and one by one through the Toeplitz path; device time of the step
    loops (pump builds excluded), 512 trajectories, FP32."""
    import torch
    pts = scan_points()
    B = 512
    t0 = time.time()
    res = twa.run_batch(pts, B, steps, precision=precision, integrator=integrator,
                        progress=max(1000, steps // 20))
    torch.cuda.synchronize()
    batch_wall = time.time() - t0
    batch_ms = res[0]["kernel_ms"]
    work = sum(B * N * steps for (N, _, _, _, _) in pts)
    flops = sum(12.0 * N * N * B * steps for (N, _, _, _, _) in pts)
    crit = [r["step_criterion"] for r in res]
    peak = PEAK_TFLOPS["bf16" if precision == "bf16x3" else precision]
    # split BF16 performs three BF16 products per contraction value: its
    # MFMA flops are 3x the algorithmic ones (the rate below is algorithmic)
    out = {"points": len(pts), "n_traj": B, "steps": steps, "precision": precision, "integrator": integrator,
           "N_list": [p[0] for p in pts], "step_criterion_min_max": [min(crit), max(crit)],
           "tile_configs": sorted(set(r["tile_config"] for r in res)),
           "batched_ms": batch_ms, "batched_rate": work / (batch_ms * 1e-3), "unit": "trajectory-atom-steps/s",
           "batched_tflops": flops / (batch_ms * 1e-3) / 1e12,
           "batched_frac_fp32_peak": flops / (batch_ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp32"],
           "batched_frac_own_peak": (3.0 if precision == "bf16x3" else 1.0) * flops / (batch_ms * 1e-3) / 1e12 / peak,
           "batch_wall_s_incl_pumps_and_tuning": batch_wall,
           "max_norm_dev_max": max(r["max_norm_dev"] for r in res)}
    if singles:
        single_ms = 0.0
        toep_ms = 0.0
        for i, (N, w, a, dt, seed) in enumerate(pts):
            p = twa.build_pump(N, w, a)
            r = twa.run(p, B, dt, steps, seed=seed, point=i, precision=precision, integrator=integrator)
            single_ms += r.obs["kernel_ms"]
            p.close()
            lt = twa.build_pump_toeplitz(N, w, a)
            t = twa.run(lt, B, dt, steps, seed=seed, point=i, precision="fp32", pump_path="toeplitz", norm_tol=-1)
            toep_ms += t.obs["kernel_ms"]
        out.update({"single_runs_ms": single_ms, "toeplitz_single_runs_ms": toep_ms,
                    "speedup_batched_vs_single": single_ms / batch_ms,
                    "speedup_toeplitz_vs_single": single_ms / toep_ms})
    return out


def batch_precision_check(twa, steps, integrator="sib"):
    """The 96-point scan for `steps` steps in FP64, FP32 and split BF16 at
    the same noise: per point the relative difference of <S+S-> and g2
    against FP64, and in units of the point's standard error; the largest
    over the points, and the device time of each."""
    pts = scan_points()
    B = 512
    runs = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        print("[bench]   scan in %s, %d steps" % (prec, steps), file=sys.stderr, flush=True)
        runs[prec] = twa.run_batch(pts, B, steps, precision=prec, integrator=integrator,
                                   progress=max(500, steps // 4))
    ref = runs["fp64"]
    out = {"points": len(pts), "n_traj": B, "steps": steps, "integrator": integrator, "modes": {}}
    for prec in ("fp32", "bf16x3"):
        rel = {k: max(abs(a[k] - b[k]) / abs(b[k]) for a, b in zip(runs[prec], ref)) for k in ("SpSm", "g2")}
        se = {k: max(abs(a[k] - b[k]) / b[k + "_se"] for a, b in zip(runs[prec], ref)) for k in ("SpSm", "g2")}
        out["modes"][prec] = {"max_rel_error_vs_fp64": rel, "max_error_vs_fp64_in_se": se,
                              "batched_ms": runs[prec][0]["kernel_ms"]}
    out["modes"]["fp64"] = {"batched_ms": ref[0]["kernel_ms"]}
    return out


def _se_shift(a, b, k):
    """difference of observable k between two runs in combined standard errors"""
    return (a[k] - b[k]) / math.sqrt(a[k + "_se"] ** 2 + b[k + "_se"] ** 2)


def heun_line(twa, pump, B, dt, T, prec, sib_obs):
    """The headline run with the stochastic Heun integrator (no spin-length
    check: its drift at this step size is the point of the comparison)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.time()
    r = twa.run(pump, B, dt, T, seed=0, precision=prec, integrator="heun", norm_tol=-1)
    torch.cuda.synchronize()
    wall = time.time() - t0
    o = r.obs
    return {"value": B * pump.N * T / wall, "unit": "trajectory-atom-steps/s", "n_steps": T,
            "ms_per_integration_step": o["kernel_ms"] / T, "max_norm_dev": o["max_norm_dev"],
            "observables": {k: o[k] for k in ("Sz", "SpSm", "g2", "Sz_se", "SpSm_se", "g2_se")},
            "shift_vs_semi_implicit_in_se": {k: _se_shift(o, sib_obs, k) for k in ("Sz", "SpSm", "g2")},
            "relative_shift_vs_semi_implicit": {k: (o[k] - sib_obs[k]) / abs(sib_obs[k]) for k in ("SpSm", "g2")}}


def precision_table(twa, pump, B, dt, integrator, T=2000):
    """The headline workload for T steps (window over the last half, same
    noise) in every contraction precision: device time per step, speed-up
    over FP32, and the error of <S^z>, <S+S-> and g2 against FP64 (relative,
    and in units of the FP64 run's standard error)."""
    out = {"n_steps": T, "integrator": integrator, "modes": {}}
    runs = {}
    for prec in ("fp64", "fp32", "bf16x3", "bf16", "fp16"):
        print("[bench]   precision %s, %d steps" % (prec, T), file=sys.stderr, flush=True)
        twa.run(pump, B, dt, 16, seed=0, precision=prec, integrator=integrator, norm_tol=-1)
        r = twa.run(pump, B, dt, T, seed=0, precision=prec, integrator=integrator, norm_tol=-1)
        runs[prec] = r.obs
    ref = runs["fp64"]
    for prec, o in runs.items():
        m = {"ms_per_step": o["kernel_ms"] / T, "speedup_vs_fp32": runs["fp32"]["kernel_ms"] / o["kernel_ms"],
             "tile_config": o["tile_config"], "max_norm_dev": o["max_norm_dev"]}
        if prec != "fp64":
            m["rel_error_vs_fp64"] = {k: abs(o[k] - ref[k]) / abs(ref[k]) for k in ("Sz", "SpSm", "g2")}
            m["error_vs_fp64_in_se"] = {k: abs(o[k] - ref[k]) / ref[k + "_se"] for k in ("Sz", "SpSm", "g2")}
        else:
            m["observables"] = {k: o[k] for k in ("Sz", "SpSm", "g2", "Sz_se", "SpSm_se", "g2_se")}
        out["modes"][prec] = m
    return out


def linewidth_precision(twa, N=1000, w=1.0, alpha=1.0, B=1024, dt=1e-4, T=4000, lags=500):
    """Linewidth (FWHM of the spectrum of the two-time correlation, from the two
    tangent-linear response copies) of the N = 1000 workload in FP64, FP32,
    split BF16, BF16 and FP16 contractions, same noise, and its error against
    FP64; Heun (the response copies are defined for it), window over the last
    half."""
    pump = twa.build_pump(N, w, alpha)
    burn = T // 2
    stride = max(1, (T - burn) // lags)
    out = {"config": {"N": N, "w": w, "alpha": alpha, "n_traj": B, "dt": dt, "n_steps": T, "burnin": burn,
                      "n_lags": lags, "lag_stride": stride}, "modes": {}}
    res = {}
    for prec in ("fp64", "fp32", "bf16x3", "bf16", "fp16"):
        r = twa.run(pump, B, dt, T, seed=0, precision=prec, burnin=burn, n_lags=lags, lag_stride=stride, norm_tol=-1)
        res[prec] = r.obs
    ref = res["fp64"]
    for prec, o in res.items():
        out["modes"][prec] = {"linewidth": o["linewidth"], "linewidth_sym": o["linewidth_sym"],
                              "ms_per_step": o["kernel_ms"] / T,
                              "rel_error_vs_fp64": abs(o["linewidth"] - ref["linewidth"]) / abs(ref["linewidth"]),
                              "max_norm_dev": o["max_norm_dev"]}
    return out


def sib_rate(twa, pump, B, dt, prec, steps=400):
    """Device time per step of the semi-implicit midpoint scheme against Heun
    on the headline pump (same three operand sweeps per step)."""
    out = {}
    for integ in ("heun", "sib"):
        twa.run(pump, B, dt, 32, seed=0, precision=prec, integrator=integ, norm_tol=-1)
        r = twa.run(pump, B, dt, steps, seed=0, precision=prec, integrator=integ, norm_tol=-1)
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
    twa.run(pump, B, dt, 64, seed=0, precision=prec, norm_tol=-1)
    plain = twa.run(pump, B, dt, T, seed=0, precision=prec, burnin=burn, norm_tol=-1).obs["kernel_ms"]
    print("[bench]   plain run %d steps: %.1f s of device time" % (T, plain / 1e3), file=sys.stderr, flush=True)
    twa.run(pump, B, dt, 64, seed=0, precision=prec, burnin=32, n_lags=16, lag_stride=2, norm_tol=-1)
    r = twa.run(pump, B, dt, T, seed=0, precision=prec, burnin=burn, n_lags=lags, lag_stride=stride, norm_tol=-1)
    lagged = r.obs["kernel_ms"]
    print("[bench]   run with %d lags: %.1f s of device time" % (lags, lagged / 1e3), file=sys.stderr, flush=True)
    per_step = plain / T
    window = (lagged - plain) / (T - burn) + per_step
    return {"config": {"N": N, "w": w, "alpha": alpha, "n_traj": B, "dt": dt, "n_steps": T, "burnin": burn,
                       "n_lags": lags, "lag_stride": stride, "precision": prec},
            "plain_ms": plain, "with_lags_ms": lagged, "plain_ms_per_step": per_step,
            "window_ms_per_step": window, "window_cost_ratio": window / per_step,
            "linewidth": r.obs.get("linewidth")}


def threshold_vs_scan(twa, N=2000, alpha=1.0, B=2048, dt=1e-4, T=2048):
    """Locating a threshold by Newton steps with pathwise gradients against
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
        r = twa.run(p, B, dt, T, seed=0, precision="fp32", burnin=burn, norm_tol=-1)
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
    fwd = float(np.median(t_fwd))
    n_bisect = int(math.ceil(math.log2((hi - lo) / tol)))
    out = {"config": {"N": N, "alpha": alpha, "n_traj": B, "dt": dt, "n_steps": T, "precision": "fp32"},
           "objective": "spsm_n", "target": target, "bracket": [lo, hi], "forward_run_s": fwd,
           "bisection_forward_runs_same_tol": n_bisect}
    # Newton with forward- or reverse-mode derivatives in FP32, and with the
    # forward mode in split BF16 (FP32-class accuracy), all against FP32
    # bisection
    for name, mode, prec in (("forward", "forward", "fp32"), ("adjoint", "adjoint", "fp32"),
                             ("forward_bf16x3", "forward", "bf16x3")):
        torch.cuda.synchronize()
        t0 = time.time()
        w_root, f_root, it = twa.find_threshold(N, alpha, B, dt, T, 0, objective="spsm_n", target=target, w_lo=lo,
                                                w_hi=hi, tol_w=tol, precision=prec, burnin=burn, norm_tol=-1,
                                                derivative=mode)
        torch.cuda.synchronize()
        el = time.time() - t0
        out[name] = {"w_root": w_root, "residual": f_root, "gradient_evaluations": it, "newton_s": el,
                     "precision": prec, "speedup_vs_bisection": n_bisect * fwd / el}
        print("[bench]   Newton (%s, %s): w = %.9g in %.1f s" % (mode, prec, w_root, el), file=sys.stderr, flush=True)
    out["forward_bf16x3"]["w_root_rel_diff_vs_fp32"] = abs(out["forward_bf16x3"]["w_root"] - out["forward"]["w_root"]) / \
        out["forward"]["w_root"]
    return out


def toeplitz_rate(twa, N, w, alpha, B, dt, T, dense_value):
    """The same workload through the circulant embedding of Eq. (2) (FFT
    drift and circulant pump noise, equal in law to the dense path), FP32
    Heun (its only integrator; no spin-length check), one full run after a
    short warm-up run."""
    import torch
    light = twa.build_pump_toeplitz(N, w, alpha)
    twa.run(light, B, dt, 256, seed=0, precision="fp32", pump_path="toeplitz", norm_tol=-1)
    torch.cuda.synchronize()
    t0 = time.time()
    r = twa.run(light, B, dt, T, seed=0, precision="fp32", pump_path="toeplitz", norm_tol=-1)
    torch.cuda.synchronize()
    wall = time.time() - t0
    value = B * N * T / wall
    M = 256
    while M < 2 * N - 2:
        M *= 2
    return {"value": value, "unit": "trajectory-atom-steps/s", "precision": "fp32", "integrator": "heun",
            "n_steps": T, "wall_s": wall, "kernel_ms": r.obs["kernel_ms"], "speedup_vs_dense": value / dense_value,
            "embedding_size": M, "max_norm_dev": r.obs["max_norm_dev"],
            "observables": {k: r.obs[k] for k in ("Sz", "SpSm", "g2", "Sz_se", "SpSm_se", "g2_se")}}


def copy_calibration():
    """One plain device copy of a known size (1 GiB read, 1 GiB written), run
    under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE to obtain the scale between
    counter readings and bytes moved."""
    import torch
    n = 1 << 28                      # 2^28 float32 = 1 GiB
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes" % (4 * n), flush=True)


def toeplitz_only(twa, N, w, alpha, B, dt):
    """Profiling workload of the Toeplitz kernel: a one-launch warm-up run of
    256 steps, then 512 steps (two launches of 256)."""
    import torch
    p = twa.build_pump_toeplitz(N, w, alpha)
    twa.run(p, B, dt, 256, seed=0, precision="fp32", pump_path="toeplitz", norm_tol=-1)
    torch.cuda.synchronize()
    t0 = time.time()
    r = twa.run(p, B, dt, 512, seed=0, precision="fp32", pump_path="toeplitz", norm_tol=-1)
    torch.cuda.synchronize()
    print("toeplitz N=%d B=%d: %.3f ms per step (kernel %.3f)" % (N, B, 1e3 * (time.time() - t0) / 512,
                                                                 r.obs["kernel_ms"] / 512), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="bench steps of 1000 integration steps each")
    ap.add_argument("--warmup", type=int, default=1, help="untimed bench steps before the timed run")
    ap.add_argument("--precision", default="bf16", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--integrator", default="sib", choices=["sib", "heun"])
    ap.add_argument("--tile-config", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-toeplitz", action="store_true")
    ap.add_argument("--no-heun", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-linewidth", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="skip every line beside the headline")
    ap.add_argument("--sib", action="store_true", help="also time the semi-implicit scheme against Heun per step")
    ap.add_argument("--threshold", action="store_true",
                    help="also time the Newton threshold searches against bisection")
    ap.add_argument("--two-time", action="store_true",
                    help="also time the two-time correlation window (N = 1000, 4096 trajectories, FP32)")
    ap.add_argument("--two-time-steps", type=int, default=4000,
                    help="with --two-time: integration steps (window over the last half)")
    ap.add_argument("--two-time-lags", type=int, default=500, help="with --two-time: number of lags")
    ap.add_argument("--adjoint-steps", type=int, default=2048,
                    help="integration steps of the adjoint cost line (N = 2000, 2048 trajectories)")
    ap.add_argument("--adjoint", action="store_true", help="the adjoint cost line also with --headline-only")
    ap.add_argument("--gradient-check", default="", choices=["", "fp32", "fp64"],
                    help="dg2/dw on the adjoint workload by forward mode and by central differences at several h "
                         "(--adjoint-steps steps) in this precision")
    ap.add_argument("--batch-scan", type=int, default=0,
                    help="also time the 96-point scan for this many steps")
    ap.add_argument("--batch-singles", action="store_true",
                    help="with --batch-scan: also run the 96 points one by one (dense and Toeplitz)")
    ap.add_argument("--batch-singles-only", type=int, default=0,
                    help="run only the 96 points one by one (dense) for this many steps")
    ap.add_argument("--batch-precision", default="fp32", choices=["fp32", "bf16x3"],
                    help="contraction precision of the batched scan and its single runs")
    ap.add_argument("--batch-precision-check", type=int, default=0,
                    help="the scan for this many steps in FP64, FP32 and split BF16: errors against FP64")
    ap.add_argument("--copy-calibration", action="store_true", help="one 1 GiB device copy, then exit")
    ap.add_argument("--toeplitz-only", action="store_true", help="the Toeplitz profiling workload, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (trajectories would shard "
              "across GPUs with one all-reduce of the accumulators at the end)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    import paper_2608_10075_amd as twa

    N, alpha, B, dt = 10000, 1.0, 1024, 1e-4
    T = STEPS_PER_BENCH_STEP * args.steps
    w = math.log(N)
    prec = args.precision
    integ = args.integrator
    if args.toeplitz_only:
        toeplitz_only(twa, N, w, alpha, B, dt)
        return
    if args.headline_only:
        args.no_cpu_baseline = args.no_toeplitz = args.no_heun = True
        args.no_adjoint = not args.adjoint
        args.no_precision = args.no_linewidth = True
    workload = "n1e4"
    print("[bench] building pump N=%d alpha=%g w=%.4f" % (N, alpha, w), file=sys.stderr, flush=True)
    t0 = time.time()
    pump = twa.build_pump(N, w, alpha)
    torch.cuda.synchronize()
    pump_s = time.time() - t0

    if args.warmup > 0:
        print("[bench] warmup: %d integration steps" % (STEPS_PER_BENCH_STEP * args.warmup), file=sys.stderr,
              flush=True)
        twa.run(pump, B, dt, STEPS_PER_BENCH_STEP * args.warmup, seed=0, precision=prec, integrator=integ,
                tile_config=args.tile_config, timing=True)
    print("[bench] timed run: %d integration steps (%d bench steps)" % (T, args.steps), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.time()
    res = twa.run(pump, B, dt, T, seed=0, precision=prec, integrator=integ, tile_config=args.tile_config,
                  timing=True, allow_unstable=(integ == "heun"))
    torch.cuda.synchronize()
    wall = time.time() - t0
    print("[bench] timed run done: %.2f s" % wall, file=sys.stderr, flush=True)
    ms_per_step = 1e3 * wall / args.steps
    value = B * N * T / wall
    o = res.obs
    flops1 = 2.0 * N * (2 * N) * (2 * B)
    flops2 = 2.0 * N * N * (2 * B)
    s1 = o["stage1_ms"] / o["stage1_launches"]
    s2 = o["stage2_ms"] / o["stage2_launches"]
    ach1 = flops1 / (s1 * 1e-3) / 1e12
    ach2 = flops2 / (s2 * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
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
        "config": {"workload": "TWA chain N=10000 alpha=1 w=ln(N) Gamma=1, 1024 trajectories, dt=1e-4, %d %s "
                               "steps (one bench step = %d integration steps), window = last half, %s "
                               "channel-mixing contraction" % (T, integ, STEPS_PER_BENCH_STEP, prec),
                   "N": N, "alpha": alpha, "w": w, "n_traj": B, "dt": dt, "n_steps": T,
                   "integration_steps_per_bench_step": STEPS_PER_BENCH_STEP, "precision": prec,
                   "integrator": integ, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": ach1, "peak": peak, "unit": "TFLOP/s", "frac": ach1 / peak,
                     "traffic": traffic_from_profiles(workload, prec, integ),
                     "kernel": "heun_stage_kernel stage 1 (predictor contraction, K = 2N)",
                     "flops_per_launch": flops1, "mean_launch_ms": s1, "launches": o["stage1_launches"]},
        "roofline_stage2": {"achieved": ach2, "peak": peak, "unit": "TFLOP/s", "frac": ach2 / peak,
                            "mean_launch_ms": s2, "flops_per_launch": flops2, "launches": o["stage2_launches"]},
        "step_ms": o["kernel_ms"] / T,
        "pump_build_s": pump_s,
        "status": res.status,
        "observables": {k: o[k] for k in ("Sz", "SpSm", "g2", "Sz_se", "SpSm_se", "g2_se", "max_norm_dev",
                                          "step_criterion")},
        "tile_config": o["tile_config"],
    }
    if not args.no_heun and integ == "sib":
        print("[bench] Heun integrator on the same workload", file=sys.stderr, flush=True)
        line["heun"] = heun_line(twa, pump, B, dt, T, prec, o)
    if not args.no_precision:
        print("[bench] precision modes vs FP64 (2000 steps)", file=sys.stderr, flush=True)
        line["precision"] = precision_table(twa, pump, B, dt, integ)
    if not args.no_linewidth:
        print("[bench] linewidth in each precision (N=1000)", file=sys.stderr, flush=True)
        line["linewidth_precision"] = linewidth_precision(twa)
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
        line["two_time"] = two_time_cost(twa, T=args.two_time_steps, lags=args.two_time_lags)
        print("[bench]   " + json.dumps(line["two_time"]), file=sys.stderr, flush=True)
    if args.batch_scan > 0:
        print("[bench] batched scan, 96 points, %d steps" % args.batch_scan, file=sys.stderr, flush=True)
        line["batch_scan"] = batch_scan(twa, args.batch_scan, singles=args.batch_singles,
                                        precision=args.batch_precision)
    if args.batch_singles_only > 0:
        print("[bench] the 96 scan points one by one, %d steps" % args.batch_singles_only, file=sys.stderr, flush=True)
        line["batch_singles"] = batch_singles(twa, args.batch_singles_only, precision=args.batch_precision)
    if args.batch_precision_check > 0:
        print("[bench] scan precision check, %d steps" % args.batch_precision_check, file=sys.stderr, flush=True)
        line["batch_precision_check"] = batch_precision_check(twa, args.batch_precision_check)
    if not args.no_adjoint:
        print("[bench] adjoint cost ratio (N=2000, FP32)", file=sys.stderr, flush=True)
        line["adjoint"] = adjoint_cost(twa, steps=args.adjoint_steps)
        print("[bench]   " + json.dumps(line["adjoint"]), file=sys.stderr, flush=True)
    if args.gradient_check:
        print("[bench] gradient check (N=2000, %s, %d steps)" % (args.gradient_check, args.adjoint_steps),
              file=sys.stderr, flush=True)
        hs = (1e-3, 1e-4, 1e-5, 1e-6) if args.gradient_check == "fp32" else (1e-5, 1e-6, 1e-7, 1e-8)
        line["gradient_check"] = gradient_check(twa, args.adjoint_steps, args.gradient_check, hs)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"], opump_ = cpu_baseline(N, w, alpha, dt, integ)
        line["cpu_baseline_single_core"], _ = cpu_baseline(N, w, alpha, dt, integ, budget_s=8.0, threads=1,
                                                           pump=opump_, B=8)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
