"""Batched scan (grouped persistent launches over many points) through the
C ABI: every point equals its own single run bit for bit, and the single
runs match the FP64 oracle (test_gpu_parity), so the scan does too."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def _points(n, seed=0, nmin=40, nmax=400):
    rng = np.random.default_rng(seed)
    Ns = rng.integers(nmin, nmax + 1, n)
    alphas = np.linspace(0.0, 3.0, 4)
    ws = np.logspace(-1, 1, 3)
    pts = []
    for i in range(n):
        a = alphas[i % 4]
        w = ws[(i // 4) % 3]
        N = int(Ns[i])
        pts.append((N, float(w), float(a), 0.02 / N, 100 + i))
    return pts


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_equals_single_runs(twa, prec, tmp_path):
    pts = _points(12)
    B, T = 40, 60
    cache = str(tmp_path / "tune.txt")
    outs = twa.run_batch(pts, B, T, precision=prec, tune_cache=cache)
    assert os.path.exists(cache) and len(open(cache).read().split()) == 2
    cfg = outs[0]["tile_config"]
    for i, (N, w, a, dt, seed) in enumerate(pts):
        p = twa.build_pump(N, w, a)
        r = twa.run(p, B, dt, T, seed=seed, point=i, precision=prec, tile_config=cfg)
        for k in ("T2", "T3", "T4", "Z", "ZZ", "SpSm", "g2", "max_norm_dev"):
            assert outs[i][k] == r.obs[k], (i, k, outs[i][k], r.obs[k])
    # a second call reads the tuned configuration from the cache
    again = twa.run_batch(pts, B, T, precision=prec, tune_cache=cache)
    assert [o["SpSm"] for o in again] == [o["SpSm"] for o in outs]


def test_batch_graph_replay_equals_direct_launches(twa):
    pts = _points(5, seed=3)
    a = twa.run_batch(pts, 32, 70, use_graph=True, steps_per_graph=8)
    b = twa.run_batch(pts, 32, 70, use_graph=False)
    assert [o["g2"] for o in a] == [o["g2"] for o in b]


def test_batch_rejects_bad_input(twa):
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, 1.0, 1.0, 1e-3, 0)], 8, 10, burnin=10)
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, -1.0, 1.0, 1e-3, 0)], 8, 10)
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, 1.0, 1.0, 1e-3, 0)], 8, 10, precision="fp64")
