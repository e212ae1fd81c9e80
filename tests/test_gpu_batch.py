"""Batched scan (grouped persistent launches over many points, one tile
configuration per N bucket, buckets on parallel stream branches) through the
C ABI: every point against the FP64 oracle per trajectory (window moments,
final states and two-time block sums), every point against its own single
run bit for bit, graph replay against direct launches, and the autotuner's
per-bucket cache."""
import functools
import os

import numpy as np
import pytest

from oracle import pump as opump
from oracle import twa as otwa

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


# one point in each N bucket (<= 128, <= 1024, larger), ragged sizes
ORACLE_POINTS = [(70, 1.0, 0.5, 2e-4, 11), (300, 2.0, 1.0, 6e-5, 12), (1100, 3.0, 1.5, 2e-5, 13)]
# and the upper end of the scan's N range in the large-N bucket
ORACLE_POINTS_WIDE = ORACLE_POINTS + [(4096, 1.5, 2.0, 5e-6, 14)]


@functools.lru_cache(maxsize=None)
def _oracle(pt, index, B, T, burnin, **kw):
    N, w, a, dt, seed = pt
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=a, n_traj=B, dt=dt, n_steps=T, seed=seed, point=index,
                         burnin=burnin, **kw)
    return otwa.run(cfg, opump.build_pump(N, w, a))


# split BF16: 1e-4, the bound of its single-run parity tests (each operand to
# 2^-17 relative, the dropped lo x lo product below 2^-18)
@pytest.mark.parametrize("prec,tile,tol", [("fp64", -1, 1e-10), ("fp32", -1, 1e-5), ("fp32", 7, 1e-5),
                                           ("fp32", 2, 1e-5), ("bf16x3", -1, 1e-4), ("bf16x3", 7, 1e-4)])
def test_batch_points_match_oracle(twa, prec, tile, tol):
    """Each point of a batch spanning the three N buckets and reaching the
    scan's largest N against the FP64 oracle per trajectory: window moments
    T2 ... ZZ and final states (tile -1: autotuned per bucket; 7 and 2: those
    tiles for every point)."""
    B, T, burn = 40, 40, 20
    res = twa.run_batch(ORACLE_POINTS_WIDE, B, T, burnin=burn, precision=prec, tile_config=tile, want_traj=True,
                        want_final_state=True, norm_tol=-1)
    for i, (pt, r) in enumerate(zip(ORACLE_POINTS_WIDE, res)):
        ref = _oracle(pt, i, B, T, burn)
        if tile >= 0:
            assert r.obs["tile_config"] == tile
        g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
        o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
        srel = np.max(np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1))
        mrel = np.max(np.abs(r.traj_moments - ref.traj_moments) / np.abs(ref.traj_moments).max(axis=0))
        print("batch %s point %d N=%d tile %d: state rel %.2e moments rel %.2e" % (
            prec, i, pt[0], r.obs["tile_config"], srel, mrel))
        assert srel < tol and mrel < tol, (i, srel, mrel)


@pytest.mark.parametrize("prec,tile,tol", [("fp64", -1, 1e-10), ("fp32", 7, 1e-5), ("bf16x3", 7, 1e-4)])
def test_batch_two_time_matches_oracle(twa, prec, tile, tol):
    """Two-time correlation of every point of the batch (response copies in
    grouped launches) against the oracle's block sums."""
    B, T, burn, L, stride = 40, 60, 36, 7, 4
    res = twa.run_batch(ORACLE_POINTS, B, T, burnin=burn, precision=prec, tile_config=tile, n_lags=L,
                        lag_stride=stride, want_lags=True, norm_tol=-1)
    for i, (pt, r) in enumerate(zip(ORACLE_POINTS, res)):
        ref = _oracle(pt, i, B, T, burn, n_lags=L, lag_stride=stride)
        corr = (r.corr_blocks[..., 0] + 1j * r.corr_blocks[..., 1]).T
        chi = r.chi_blocks.transpose(1, 2, 0)
        ec = np.max(np.abs(corr - ref.corr_blocks)) / np.abs(ref.corr_blocks).max()
        ex = np.max(np.abs(chi - ref.chi_blocks)) / np.abs(ref.chi_blocks).max()
        print("batch two-time %s point %d tile %d: corr rel %.2e chi rel %.2e" % (prec, i, r.obs["tile_config"],
                                                                                 ec, ex))
        assert ec < tol and ex < tol, (i, ec, ex)
        assert r.obs["n_lags"] == L and r.obs["lag_stride"] == stride


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
def test_batch_equals_single_runs(twa, prec, tmp_path):
    pts = _points(9) + [(1300, 1.0, 1.0, 2e-5, 500)]
    B, T = 40, 60
    cache = str(tmp_path / "tune.txt")
    outs = twa.run_batch(pts, B, T, precision=prec, tune_cache=cache, norm_tol=-1)
    # one cache line per N bucket that holds points
    buckets = {0 if N <= 128 else 1 if N <= 1024 else 2 for (N, _, _, _, _) in pts}
    assert os.path.exists(cache) and len(open(cache).read().split()) == 2 * len(buckets)
    for i, (N, w, a, dt, seed) in enumerate(pts):
        p = twa.build_pump(N, w, a)
        r = twa.run(p, B, dt, T, seed=seed, point=i, precision=prec, tile_config=outs[i]["tile_config"],
                    norm_tol=-1)
        for k in ("T2", "T3", "T4", "Z", "ZZ", "SpSm", "g2", "max_norm_dev"):
            assert outs[i][k] == r.obs[k], (i, k, outs[i][k], r.obs[k])
    # a second call reads the tuned configurations from the cache
    again = twa.run_batch(pts, B, T, precision=prec, tune_cache=cache, norm_tol=-1)
    assert [o["SpSm"] for o in again] == [o["SpSm"] for o in outs]
    assert [o["tile_config"] for o in again] == [o["tile_config"] for o in outs]


def test_batch_graph_replay_equals_direct_launches(twa):
    pts = _points(5, seed=3) + [(1100, 2.0, 1.0, 2e-5, 77)]
    kw = dict(norm_tol=-1, n_lags=4, lag_stride=3, burnin=40)
    a = twa.run_batch(pts, 32, 70, use_graph=True, steps_per_graph=8, **kw)
    b = twa.run_batch(pts, 32, 70, use_graph=False, **kw)
    assert [o["g2"] for o in a] == [o["g2"] for o in b]
    assert [o["linewidth_sym"] for o in a] == [o["linewidth_sym"] for o in b]


def test_batch_rejects_bad_input(twa):
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, 1.0, 1.0, 1e-3, 0)], 8, 10, burnin=10)
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, -1.0, 1.0, 1e-3, 0)], 8, 10)
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, 1.0, 1.0, 1e-3, 0)], 8, 10, precision="bf16x3", tile_config=5)
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, 1.0, 1.0, 1e-3, 0)], 8, 10, tile_config=7, precision="fp64")
    with pytest.raises(twa.TWAError):
        twa.run_batch([(10, 1.0, 1.0, 1e-3, 0)], 8, 10, n_lags=4, integrator="sib")
