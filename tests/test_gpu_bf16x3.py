"""Split-BF16 contractions (TWA_PREC_BF16X3: operands as bf16 hi + lo, the
product as Ahi Xhi + Ahi Xlo + Alo Xhi on BF16 MFMA) through the C ABI
against the FP64 oracle.

Tolerance: each operand value is represented to 2^-17 relative (hi, then lo
of the remainder) and the dropped Alo Xlo term is below 2^-18 of |A||X|, so a
contracted field increment carries about 2^-16 relative error, against
2^-8 for plain BF16.  With per-step field increments of a few percent of a
spin (dt = 0.02 / N here) accumulated without cancellation over 200 steps,
states stay within 1e-4 relative per trajectory; the test also checks the
error is at least 20x below plain BF16's on the same run."""
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


def _oracle(N, w, alpha, B, dt, T, seed, **kw):
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=seed, **kw)
    return otwa.run(cfg, opump.build_pump(N, w, alpha))


def _relerr(r, ref, B):
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    return (np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)).max()


@pytest.mark.parametrize("N,B,cfg,integ", [(300, 70, 2, "heun"), (650, 130, 7, "heun"), (257, 40, 3, "heun"),
                                           (300, 33, 2, "sib"), (100, 20, -1, "heun")])
def test_split_bf16_matches_oracle(twa, N, B, cfg, integ):
    w, alpha, T, seed = 2.0, 1.0, 200, 4
    dt = 0.02 / N
    p = twa.build_pump(N, w, alpha)
    r3 = twa.run(p, B, dt, T, seed=seed, precision="bf16x3", tile_config=cfg, integrator=integ,
                 want_final_state=True, want_traj=True, norm_tol=-1)
    r1 = twa.run(p, B, dt, T, seed=seed, precision="bf16", tile_config=cfg, integrator=integ, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, seed, integrator=integ)
    e3, e1 = _relerr(r3, ref, B), _relerr(r1, ref, B)
    print("N=%d cfg %d %s: split-BF16 %.2e, BF16 %.2e" % (N, r3.obs["tile_config"], integ, e3, e1))
    assert e3 < 1e-4
    assert e3 < e1 / 20
    scale = np.abs(ref.traj_moments).max(axis=0)
    assert np.max(np.abs(r3.traj_moments - ref.traj_moments) / scale) < 1e-4


def test_split_bf16_headline_size_sampled(twa):
    """N = 1e4, 1024 trajectories (the 320 x 256 tiles): three trajectories
    re-integrated by the oracle alone."""
    N, B, T = 10000, 1024, 12
    w, alpha, dt = float(np.log(N)), 1.0, 1e-4
    r = twa.run(twa.build_pump(N, w, alpha), B, dt, T, seed=0, precision="bf16x3", want_final_state=True, norm_tol=-1)
    idx = np.array([0, 517, 1023])
    ref = _oracle(N, w, alpha, 3, dt, T, 0, traj=idx)
    for j, k in enumerate(idx):
        got = r.final_state[:, k, :]
        want = np.stack([ref.final_state[c][j] for c in range(3)])
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-4


def test_split_bf16_rejections(twa):
    p = twa.build_pump(64, 1.0, 1.0)
    with pytest.raises(twa.TWAError):
        twa.run(p, 8, 1e-3, 20, precision="bf16x3", pump_path="toeplitz", norm_tol=-1)
    W = p.matrix("W")
    model = twa.build_model(W, 0.5 * np.eye(64))
    with pytest.raises(twa.TWAError):
        twa.run(model, 8, 1e-3, 20, precision="bf16x3", norm_tol=-1)
