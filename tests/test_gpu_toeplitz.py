"""The Toeplitz fast path (circulant embedding of Eq. (2), FFT drift and
circulant pump noise, one workgroup per trajectory) through the C ABI
against the oracle's Toeplitz mode: every embedding size from 256 to 32768
points (FP32) and to 16384 (FP64), ragged N including N = 1 and the largest
N, partial chunks of steps; equal in law to the dense path; error paths."""
import numpy as np
import pytest

from oracle import observables as oobs
from oracle import toeplitz as otoe
from oracle import twa as otwa

pytestmark = pytest.mark.gpu
TOEPLITZ = 98


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def _oracle(N, w, alpha, B, dt, T, seed, **kw):
    return otwa.run(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=seed, toeplitz=True,
                                   **kw))


# (N, B, T): embedding sizes 256 (N = 1, 2, 40, 129), 512, 1024, 2048, 4096, 8192, 16384
@pytest.mark.parametrize("N,B,T", [(1, 3, 40), (2, 5, 40), (40, 17, 300), (129, 9, 120), (200, 6, 80),
                                   (513, 5, 60), (1000, 4, 40), (2049, 3, 30), (4000, 2, 20), (8193, 2, 12)])
def test_fp64_matches_oracle(twa, N, B, T):
    w, alpha, seed = 2.0, 0.8, 3
    dt = 0.02 / max(N, 50)
    p = twa.build_pump_toeplitz(N, w, alpha) if N > 1000 else twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=seed, precision="fp64", pump_path="toeplitz",
                want_traj=True, want_final_state=True, s0z=-1.0 if N % 2 else 1.0, norm_tol=-1)
    assert r.obs["tile_config"] == TOEPLITZ
    ref = _oracle(N, w, alpha, B, dt, T, seed, s0z=-1.0 if N % 2 else 1.0)
    for c in range(3):
        assert np.max(np.abs(r.final_state[c] - ref.final_state[c])) < 1e-11
    scale = np.abs(ref.traj_moments).max(axis=0) + 1e-300
    assert np.max(np.abs(r.traj_moments - ref.traj_moments) / scale) < 1e-10


@pytest.mark.parametrize("N,B,T", [(300, 8, 300), (3000, 4, 40), (6000, 3, 20), (10000, 2, 12), (16385, 2, 8)])
def test_fp32_matches_oracle(twa, N, B, T):
    w, alpha, seed = np.log(N) + 1.0, 1.0, 5
    dt = 0.02 / N
    r = twa.run(twa.build_pump_toeplitz(N, w, alpha), B, dt, T, seed=seed, precision="fp32", pump_path="toeplitz",
                want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, seed)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    assert (np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)).max() < 1e-5


def test_chunks_and_determinism(twa):
    """600 steps run as three launches of up to 256 steps; the result does
    not depend on the chunking and repeats bit for bit."""
    N, B = 300, 6
    p = twa.build_pump(N, 1.5, 1.2)
    a = twa.run(p, B, 1e-4, 600, seed=2, precision="fp64", pump_path="toeplitz", want_final_state=True,
                want_traj=True, norm_tol=-1)
    b = twa.run(p, B, 1e-4, 600, seed=2, precision="fp64", pump_path="toeplitz", want_final_state=True,
                want_traj=True, norm_tol=-1)
    assert np.array_equal(a.final_state, b.final_state) and np.array_equal(a.traj_moments, b.traj_moments)
    ref = _oracle(N, 1.5, 1.2, B, 1e-4, 600, 2)
    assert np.max(np.abs(a.final_state - np.stack(ref.final_state))) < 1e-11


def test_equal_in_law_to_the_dense_path(twa):
    """Different noise realisations of the same law: the ensemble observables
    of the two paths agree within their statistical errors."""
    N, B, T = 500, 2048, 3000
    p = twa.build_pump(N, 1.2 * N / 10.0, 0.5)
    d = twa.run(p, B, 0.02 / N, T, seed=1, precision="fp32", norm_tol=-1)
    t = twa.run(p, B, 0.02 / N, T, seed=1, precision="fp32", pump_path="toeplitz", norm_tol=-1)
    for k in ("Sz", "SpSm", "g2"):
        se = np.hypot(d.obs[k + "_se"], t.obs[k + "_se"])
        assert abs(d.obs[k] - t.obs[k]) < 5 * se, (k, d.obs[k], t.obs[k], se)


def test_observables_match_oracle_finaliser(twa):
    N, B, T = 64, 96, 400
    r = twa.run(twa.build_pump(N, 3.0, 1.0), B, 1e-3, T, seed=0, precision="fp64", pump_path="toeplitz", norm_tol=-1)
    ref = _oracle(N, 3.0, 1.0, B, 1e-3, T, 0)
    o = oobs.finalize(ref.traj_moments)
    for k in ("SpSm", "g2", "Sz", "SpSm_se", "g2_se"):
        assert abs(r.obs[k] - o[k]) <= 1e-9 * max(1.0, abs(o[k])), k


def test_light_handle(twa):
    """The Toeplitz-only handle: lam_max of the circulant bounds the channel
    rates from above; dense consumers reject it."""
    N = 300
    light, dense = twa.build_pump_toeplitz(N, 2.0, 0.7), twa.build_pump(N, 2.0, 0.7)
    tp = otoe.ToeplitzPump(N, 2.0, 0.7)
    assert abs(light.lam_max - tp.lam.max()) < 1e-10 * tp.lam.max()
    assert light.lam_max >= dense.lam_max * (1 - 1e-12) and np.isnan(light.lam_min)
    with pytest.raises(twa.TWAError):
        twa.run(light, 4, 1e-3, 10, precision="fp32", norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.protocol(light, 1.0, 0.04)
    with pytest.raises(twa.TWAError):
        light.matrix("W")
    a = twa.run(light, 4, 1e-3, 30, seed=1, precision="fp64", pump_path="toeplitz", want_final_state=True, norm_tol=-1)
    b = twa.run(dense, 4, 1e-3, 30, seed=1, precision="fp64", pump_path="toeplitz", want_final_state=True, norm_tol=-1)
    assert np.array_equal(a.final_state, b.final_state)


def test_errors(twa):
    p = twa.build_pump(50, 1.0, 1.0)
    for kw in (dict(precision="bf16"), dict(precision="fp32", n_lags=4), dict(precision="fp64", integrator="sib")):
        with pytest.raises(twa.TWAError):
            twa.run(p, 4, 1e-3, 10, pump_path="toeplitz", **kw, norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.run(twa.build_pump_toeplitz(8194, 1.0, 1.0), 2, 1e-4, 2, precision="fp64", pump_path="toeplitz", norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.build_pump_toeplitz(16386, 1.0, 1.0)
    W = np.eye(50)
    with pytest.raises(twa.TWAError):
        twa.run(twa.Pump(50, dense=W), 4, 1e-3, 10, precision="fp32", pump_path="toeplitz", norm_tol=-1)
