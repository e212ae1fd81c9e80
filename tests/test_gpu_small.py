"""The fused small-N kernel (every step of a short chain in one launch)
through the C ABI against the FP64 oracle: FP64 and FP32, Heun and the
semi-implicit scheme, ragged N (odd, one spin, up to 64) and trajectory
counts that leave partial blocks, and against the multi-kernel path."""
import numpy as np
import pytest

from oracle import pump as opump
from oracle import twa as otwa

pytestmark = pytest.mark.gpu
FUSED = 99


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def _oracle(N, w, alpha, B, dt, T, seed, **kw):
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=seed, **kw)
    return otwa.run(cfg, opump.build_pump(N, w, alpha))


@pytest.mark.parametrize("N,B,integ", [(1, 3, "heun"), (7, 5, "heun"), (16, 40, "heun"), (33, 9, "heun"),
                                       (64, 17, "heun"), (13, 21, "sib"), (50, 6, "sib")])
def test_fused_fp64_matches_oracle(twa, N, B, integ):
    w, alpha, dt, T, seed = 2.5, 0.9, 1e-3, 300, 4
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=seed, precision="fp64", s0z=-1.0, integrator=integ, want_traj=True,
                want_final_state=True, norm_tol=-1)
    assert r.obs["tile_config"] == FUSED
    ref = _oracle(N, w, alpha, B, dt, T, seed, s0z=-1.0, integrator=integ)
    for c in range(3):
        assert np.max(np.abs(r.final_state[c] - ref.final_state[c])) < 1e-11
    scale = np.abs(ref.traj_moments).max(axis=0) + 1e-300
    assert np.max(np.abs(r.traj_moments - ref.traj_moments) / scale) < 1e-10


@pytest.mark.parametrize("N,B", [(16, 64), (45, 30)])
def test_fused_fp32_matches_oracle(twa, N, B):
    w, alpha, T, seed = 2.0, 1.0, 1000, 5
    dt = 0.02 / N
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=seed, precision="fp32", want_final_state=True, norm_tol=-1)
    assert r.obs["tile_config"] == FUSED
    ref = _oracle(N, w, alpha, B, dt, T, seed)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    assert (np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)).max() < 1e-5


def test_fused_equals_multi_kernel_path(twa):
    N, B, w, alpha, dt, T = 24, 100, 3.0, 1.2, 1e-3, 500
    p = twa.build_pump(N, w, alpha)
    a = twa.run(p, B, dt, T, seed=9, precision="fp64", want_final_state=True, norm_tol=-1)
    b = twa.run(p, B, dt, T, seed=9, precision="fp64", tile_config=0, want_final_state=True, norm_tol=-1)
    assert a.obs["tile_config"] == FUSED and b.obs["tile_config"] == 0
    assert np.max(np.abs(a.final_state - b.final_state)) < 1e-11
    for k in ("SpSm", "g2", "Sz", "T4"):
        assert abs(a.obs[k] - b.obs[k]) <= 1e-10 * max(1.0, abs(b.obs[k])), k
