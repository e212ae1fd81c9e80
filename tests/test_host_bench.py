"""Host logic of the measurement harness (no GPU): the scan's point recipe and
step criterion, the rule that keeps counter traffic only for the kernel
source it was taken on, the one-GPU guard, the profiling commands quoted in
profiles/ (every bench.py flag they use exists), and the option defaults of
the C ABI that need no device."""
import ctypes
import glob
import importlib.util
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_scan_points_recipe(bench):
    pts = bench.scan_points()
    assert len(pts) == 96
    Ns = np.random.default_rng(0).integers(64, 4097, 96)
    alphas, ws = np.linspace(0.0, 3.0, 12), np.logspace(-2, 2, 8)
    for q, (N, w, a, dt, seed) in enumerate(pts):
        assert N == int(Ns[q]) and 64 <= N <= 4096 and seed == q
        assert a == float(alphas[q // 8]) and w == float(ws[q % 8])
        # the step criterion 0.04 / max(Gamma N, lam_max) with lam_max bounded
        # by the largest row sum of Eq. (2), computed here by brute force
        W = w / (1.0 + np.abs(np.arange(N)[:, None] - np.arange(N)[None, :])) ** a if N <= 600 else None
        if W is not None:
            bound = W.sum(axis=1).max()
            assert np.linalg.eigvalsh(W).max() <= bound * (1 + 1e-12)
            assert dt == pytest.approx(0.04 / max(N, bound), rel=1e-12)
        assert dt * N <= 0.04 * (1 + 1e-12)


def test_traffic_is_kept_only_for_the_profiled_source(bench, monkeypatch):
    path = os.path.join(ROOT, "profiles", "stage1_traffic_n1e4_bf16_sib.json")
    d = json.load(open(path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: d["source_sha"])
    assert bench.traffic_from_profiles("n1e4", "bf16", "sib") == d["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.traffic_from_profiles("n1e4", "bf16", "sib") is None
    assert bench.traffic_from_profiles("n1e4", "fp64", "sib") is None     # no such summary


def test_traffic_summary_is_per_launch_and_calibrated():
    d = json.load(open(os.path.join(ROOT, "profiles", "stage1_traffic_n1e4_bf16_sib.json")))
    cal = d["copy_calibration"]
    assert cal["fetch_scale"] == pytest.approx(cal["bytes_read"] / (cal["fetch_kib"] * 1024))
    s1 = d["stage1"]
    assert s1["read_bytes_per_launch"] == pytest.approx(s1["fetch_kib_per_launch_raw"] * 1024 * cal["fetch_scale"])
    assert d["bytes_per_launch"] == pytest.approx(s1["read_bytes_per_launch"] + s1["write_bytes_per_launch"])
    # at least the algorithmic operand stream (A once, X once) of one launch
    assert d["bytes_per_launch"] > 0.5e9


def test_stage_kernel_summaries_share_one_source():
    """Every committed summary of the contraction kernels (trace, counters,
    traffic, the equal-accuracy trace) names the kernel source it was taken
    on, and all of them name the same one: a partial re-profile fails here."""
    shas = {json.load(open(os.path.join(ROOT, "profiles", "stage1_traffic_n1e4_bf16_sib.json")))["source_sha"]}
    for f in glob.glob(os.path.join(ROOT, "profiles", "stage_kernels_*.md")):
        m = re.findall(r"Source hash[^`]*`([0-9a-f]{16})`", open(f).read())
        assert m, f
        shas |= set(m)
    assert len(shas) == 1, shas


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_profile_commands_use_existing_bench_flags():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    known = set(re.findall(r"(--[a-z][a-z0-9-]*)", r.stdout))
    texts = [open(f).read() for f in glob.glob(os.path.join(ROOT, "profiles", "*.md"))]
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.json")):
        texts += json.load(open(f)).get("commands", [])
    used = set()
    for t in texts:
        for cmd in re.findall(r"bench\.py([^\n`\"]*)", t):
            used |= set(re.findall(r"(--[a-z][a-z0-9-]*)", cmd))
    assert used, "no bench.py command found under profiles/"
    assert used <= known, used - known


def test_option_defaults_need_no_device():
    import paper_2608_10075_amd as twa
    o = twa._BatchOpts()
    twa._lib.twa_batch_opts_default(ctypes.byref(o))
    assert o.n_traj == 512 and o.burnin == -1 and o.precision == twa.PRECISIONS["fp32"]
    assert o.use_graph == 1 and o.tile_config == -1 and o.n_lags == 0
    p = twa._Params()
    twa._lib.twa_params_default(ctypes.byref(p))
    assert p.norm_tol == pytest.approx(1e-2) and p.tile_config == -1 and p.integrator == twa.INTEGRATORS["heun"]
    t = twa._ThresholdOpts()
    twa._lib.twa_threshold_opts_default(ctypes.byref(t))
    assert t.derivative == twa.DERIVATIVES["forward"]
