"""twa_build_pump_dense (an arbitrary symmetric PSD pump, the general pump the
paper's Perspectives allow at unchanged cost) against the oracle's dense pump:
the handle's matrices and channel rates, and FP64 / FP32 trajectories driven
by it, at fixed Philox noise.  Inputs: random PSD matrices of full and
deficient rank (seeded), plus the error paths."""
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


def _random_psd(n, rank, seed, scale=2.0):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, rank))
    W = scale * (G @ G.T) / rank
    return 0.5 * (W + W.T)


@pytest.mark.parametrize("n,rank", [(1, 1), (50, 50), (50, 7), (129, 129)])
def test_dense_pump_handle_matches_oracle(twa, n, rank):
    W = _random_psd(n, rank, seed=n + rank)
    p = twa.Pump(n, dense=W)
    ref = opump.build_pump_dense(W)
    assert np.array_equal(p.matrix("W"), W)
    F = p.matrix("F")
    assert np.max(np.abs(F - ref.F)) <= 1e-11 * max(1.0, np.sqrt(ref.lam_max))
    assert np.max(np.abs(F @ F - W)) <= 1e-10 * ref.lam_max
    assert abs(p.lam_max - ref.lam_max) <= 1e-12 * ref.lam_max
    assert abs(p.lam_min - ref.lam_min) <= 1e-11 * ref.lam_max


@pytest.mark.parametrize("prec,n,B,cfg,tol", [("fp64", 50, 24, 0, 1e-11), ("fp64", 129, 40, 2, 1e-11),
                                               ("fp32", 200, 70, 2, 1e-5)])
def test_dense_pump_trajectories_match_oracle(twa, prec, n, B, cfg, tol):
    W = _random_psd(n, max(3, n // 4), seed=7 * n)
    p = twa.Pump(n, dense=W)
    ref_pump = opump.build_pump_dense(W)
    dt, T, seed = 0.02 / max(n, ref_pump.lam_max), 200, 9
    r = twa.run(p, B, dt, T, seed=seed, precision=prec, tile_config=cfg, want_final_state=True, want_traj=True)
    ref = otwa.run(otwa.RunConfig(n_spin=n, w=float("nan"), alpha=float("nan"), n_traj=B, dt=dt, n_steps=T,
                                  seed=seed), ref_pump)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    rel = np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)
    mrel = np.max(np.abs(r.traj_moments - ref.traj_moments) / np.abs(ref.traj_moments).max(axis=0))
    print("dense pump %s N=%d tile %d: state rel %.2e moments rel %.2e" % (prec, n, cfg, rel.max(), mrel))
    assert rel.max() < tol and mrel < 10 * tol


def test_dense_pump_rejects_bad_matrices(twa):
    n = 20
    W = _random_psd(n, n, seed=1)
    bad = W.copy()
    bad[0, 1] += 1e-3            # not symmetric
    with pytest.raises(twa.TWAError):
        twa.Pump(n, dense=bad)
    neg = W - 2.0 * np.eye(n) * np.linalg.eigvalsh(W).max()   # negative definite
    with pytest.raises(twa.TWAError) as e:
        twa.Pump(n, dense=neg)
    assert e.value.code == twa.TWA_ENOTPSD
    nan = W.copy()
    nan[3, 3] = np.nan
    with pytest.raises(twa.TWAError):
        twa.Pump(n, dense=nan)
