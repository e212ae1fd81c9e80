"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every input is seeded: the Philox stream of the method itself (same counter
layout on both sides, implemented independently), or states from
``tests/inputs.py``.  Tolerances:
  * integer work (Philox words): bit-exact;
  * FP64 path: 1e-10 relative-to-scale (rounding order only differs);
  * FP32 path: 1e-5 relative per trajectory over 1e3 steps;
  * BF16/FP16: stated error against FP64 (no parity claim).
Parity at fixed noise holds whatever the spin-length drift of the integrator,
so these runs switch the drift check off (norm_tol=-1); the check itself
(TWA_EUNSTABLE beyond norm_tol, default 1e-2) is tested in
test_norm_drift_flag.
"""
import numpy as np
import pytest

from oracle import observables as oobs
from oracle import philox as ophilox
from oracle import pump as opump
from oracle import twa as otwa
from tests import inputs

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


def test_philox_bitwise(twa, golden_dir):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(1 << 20, 4), dtype=np.uint64).astype(np.uint32)
    out = twa.philox(ctr, 0x12345678, 0x9ABCDEF0)
    ref = ophilox.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], 0x12345678, 0x9ABCDEF0)
    assert np.array_equal(out, np.stack(ref, axis=1))
    import os
    rows = [[int(t, 16) for t in l.split()] for l in open(os.path.join(golden_dir, "philox_kat.txt"))
            if l.strip() and not l.startswith("#")]
    for r in rows:
        o = twa.philox(np.array([r[:4]], dtype=np.uint32), r[4], r[5])
        assert [int(v) for v in o[0]] == r[6:]


@pytest.mark.parametrize("N,B", [(1, 1), (7, 5), (64, 33)])
def test_noise_matches_oracle(twa, N, B):
    seed, step, point = 0xDEADBEEF12345, 17, 3
    (zx, zy), (gx, gy) = twa.noise(seed, step, B, N, point=point, fp64=True)
    rzx, rzy = ophilox.pump_noise(seed, step, B, N, point)
    rgx, rgy = ophilox.collective_noise(seed, step, B, point)
    for a, b in ((zx, rzx), (zy, rzy), (gx, rgx), (gy, rgy)):
        assert np.max(np.abs(a - b)) < 1e-13
    (fx, fy), (hx, hy) = twa.noise(seed, step, B, N, point=point, fp64=False)
    for a, b in ((fx, rzx), (fy, rzy), (hx, rgx), (hy, rgy)):
        assert np.max(np.abs(a - b) / (1.0 + np.abs(b))) < 2e-6


@pytest.mark.parametrize("N,w,alpha", [(1, 2.0, 1.0), (9, 4.0, 0.0), (37, 1.3, 0.5), (200, 2.0, 1.0), (64, 1.0, 60.0)])
def test_pump_factor_matches_oracle(twa, N, w, alpha):
    p = twa.build_pump(N, w, alpha)
    ref = opump.build_pump(N, w, alpha)
    W, F = p.matrix("W"), p.matrix("F")
    assert np.max(np.abs(W - ref.W)) <= 1e-15 * w
    assert np.max(np.abs(F - ref.F)) <= 1e-11 * max(1.0, np.sqrt(ref.lam_max))
    assert abs(p.lam_max - ref.lam_max) <= 1e-12 * ref.lam_max
    assert abs(p.lam_min - ref.lam_min) <= 1e-12 * ref.lam_max


@pytest.mark.parametrize("N,B,cfg", [(16, 32, 0), (37, 19, 0), (37, 19, 1), (130, 70, 1), (130, 70, 2), (130, 70, 3)])
def test_fp64_trajectories_match_oracle(twa, N, B, cfg):
    w, alpha, dt, T, seed = 3.0, 1.0, 1e-3, 120, 11
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=seed, precision="fp64", tile_config=cfg, s0z=-1.0,
                want_traj=True, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, seed, s0z=-1.0)
    for c in range(3):
        assert np.max(np.abs(r.final_state[c] - ref.final_state[c])) < 1e-11
    scale = np.abs(ref.traj_moments).max(axis=0) + 1e-300
    assert np.max(np.abs(r.traj_moments - ref.traj_moments) / scale) < 1e-10


@pytest.mark.parametrize("N,B,cfg", [(100, 48, 1), (100, 48, 2), (257, 40, 3), (257, 40, 4), (300, 70, 5), (300, 70, 6),
                                     (650, 130, 7), (650, 130, 8)])
def test_fp32_trajectories_1e3_steps(twa, N, B, cfg):
    """FP32 per-trajectory parity at fixed noise over 1e3 steps: 1e-5 relative,
    at a step meeting the paper's criterion max(Gamma N, w_max) dt < 0.05."""
    w, alpha, seed = 2.0, 1.0, 5
    T = 1000
    dt = 0.02 / N
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=seed, precision="fp32", tile_config=cfg, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, seed)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    rel = np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)
    assert rel.max() < 1e-5, rel.max()


def test_custom_initial_state_single_step(twa):
    N, B = 45, 21
    init = inputs.random_spins(7, B, N)
    w, alpha, dt = 2.5, 0.7, 2e-3
    p = twa.build_pump(N, w, alpha)
    for prec, tol in (("fp64", 1e-13), ("fp32", 2e-6)):
        r = twa.run(p, B, dt, 1, seed=4, precision=prec, init_state=init, want_final_state=True, norm_tol=-1)
        ref = _oracle(N, w, alpha, B, dt, 1, 4, init_state=tuple(init))
        for c in range(3):
            assert np.max(np.abs(r.final_state[c] - ref.final_state[c])) < tol


def test_two_time_fp64_matches_oracle(twa):
    N, B, w, alpha, dt, T, seed = 10, 40, 2.0, 1.0, 1e-3, 400, 2
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=seed, precision="fp64", burnin=200, n_lags=20, lag_stride=10,
                want_lags=True, want_traj=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, seed, burnin=200, n_lags=20, lag_stride=10)
    corr = r.corr_blocks[..., 0] + 1j * r.corr_blocks[..., 1]          # (L, J)
    assert np.max(np.abs(corr.T - ref.corr_blocks)) < 1e-9 * np.abs(ref.corr_blocks).max()
    chi = r.chi_blocks.transpose(1, 2, 0)                                # (J, 4, L)
    assert np.max(np.abs(chi - ref.chi_blocks)) < 1e-9 * np.abs(ref.chi_blocks).max()
    # host finaliser: linewidth of the combined correlation, same estimator as the oracle's
    csym, chiv, c = oobs.two_time(ref.corr_blocks, ref.chi_blocks, B)
    om, S = oobs.spectrum(c, 10 * dt)
    lw = oobs.fwhm(om, S)
    assert np.isfinite(r.obs["linewidth"])
    assert abs(r.obs["linewidth"] - lw) < 1e-6 * abs(lw)


def test_two_time_fp32(twa):
    N, B, w, alpha, dt, T, seed = 40, 48, 2.0, 1.0, 5e-4, 600, 9
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=seed, precision="fp32", burnin=300, n_lags=30, lag_stride=10, want_lags=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, seed, burnin=300, n_lags=30, lag_stride=10)
    corr = (r.corr_blocks[..., 0] + 1j * r.corr_blocks[..., 1]).T
    assert np.max(np.abs(corr - ref.corr_blocks)) < 1e-5 * np.abs(ref.corr_blocks).max()
    chi = r.chi_blocks.transpose(1, 2, 0)
    assert np.max(np.abs(chi - ref.chi_blocks)) < 1e-5 * np.abs(ref.chi_blocks).max()


@pytest.mark.parametrize("prec,tol,cfg", [("bf16", 3e-2, -1), ("fp16", 5e-3, -1), ("bf16", 3e-2, 3),
                                          ("bf16", 3e-2, 4), ("bf16", 3e-2, 5), ("bf16", 3e-2, 6),
                                          ("bf16", 3e-2, 7), ("fp16", 5e-3, 8)])
def test_reduced_precision_error_is_bounded(twa, prec, tol, cfg):
    N, B, w, alpha, T = (128, 64, 2.0, 1.0, 200) if cfg < 7 else (400, 150, 2.0, 1.0, 100)
    dt = 0.02 / N
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=1, precision=prec, tile_config=cfg, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, 1)
    err = max(np.max(np.abs(r.final_state[c] - ref.final_state[c])) for c in range(3))
    assert err < tol, err


def test_observables_match_oracle_finaliser(twa):
    N, B, w, alpha, dt, T = 16, 64, 4.0, 1.0, 1e-3, 600
    p = twa.build_pump(N, w, alpha)
    r = twa.run(p, B, dt, T, seed=0, precision="fp64", s0z=-1.0, norm_tol=-1)
    ref = _oracle(N, w, alpha, B, dt, T, 0, s0z=-1.0)
    o = oobs.finalize(ref.traj_moments)
    for k in ("Sz", "SpSm", "g2", "T2", "T3", "T4", "Z", "ZZ", "g2_se", "SpSm_se"):
        assert abs(r.obs[k] - o[k]) <= 1e-9 * max(1.0, abs(o[k])), k


def test_determinism_and_graph_replay(twa):
    N, B, T = 70, 36, 100
    p = twa.build_pump(N, 1.5, 0.8)
    a = twa.run(p, B, 1e-3, T, seed=8, use_graph=True, want_final_state=True, n_lags=5, lag_stride=8,
                burnin=40, want_lags=True, norm_tol=-1)
    b = twa.run(p, B, 1e-3, T, seed=8, use_graph=False, want_final_state=True, n_lags=5, lag_stride=8,
                burnin=40, want_lags=True, norm_tol=-1)
    c = twa.run(p, B, 1e-3, T, seed=8, use_graph=True, want_final_state=True, n_lags=5, lag_stride=8,
                burnin=40, want_lags=True, norm_tol=-1)
    assert np.array_equal(a.final_state, b.final_state) and np.array_equal(a.final_state, c.final_state)
    assert np.array_equal(a.corr_blocks, b.corr_blocks) and np.array_equal(a.chi_blocks, c.chi_blocks)


def test_edge_cases(twa):
    p = twa.build_pump(1, 2.0, 1.0)
    r = twa.run(p, 1, 1e-3, 50, seed=1, precision="fp64", want_final_state=True, norm_tol=-1)
    ref = _oracle(1, 2.0, 1.0, 1, 1e-3, 50, 1)
    assert np.max(np.abs(r.final_state - np.stack(ref.final_state))) < 1e-12
    p = twa.build_pump(5, 1.0, 1.0)
    r = twa.run(p, 3, 1e-3, 0, seed=1, want_final_state=True, allow_unstable=True, norm_tol=-1)
    x, y, z = otwa.initial_state(1, 3, 5)
    assert np.array_equal(r.final_state, np.stack([x, y, z]))
    with pytest.raises(twa.TWAError):
        twa.run(p, 3, 1e-3, 10, burnin=11, norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.run(p, 3, 1e-3, 10, burnin=5, n_lags=4, lag_stride=2, norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.run(p, 0, 1e-3, 10, norm_tol=-1)


def test_norm_drift_flag(twa):
    """Eq. (S1) conserves every |s_i|^2: a run whose spin lengths drift past
    norm_tol (default 1e-2) returns TWA_EUNSTABLE with its outputs written;
    the semi-implicit scheme keeps the lengths and passes the default check.
    Workload: the FP64 configuration (N = 16, alpha = 1, w = 4, atoms down,
    dt = 1e-3) over 4000 steps, where Heun drifts by a few percent; the fused
    small-N kernel, the multi-kernel path (tile 0), the adjoint and the batch."""
    N, B, w, alpha, dt, T = 16, 32, 4.0, 1.0, 1e-3, 4000
    p = twa.build_pump(N, w, alpha)
    for cfg in (-1, 0):
        with pytest.raises(twa.TWAError) as e:
            twa.run(p, B, dt, T, seed=1, precision="fp64", s0z=-1.0, tile_config=cfg)
        assert e.value.code == twa.TWA_EUNSTABLE and "drifted" in str(e.value)
        r = twa.run(p, B, dt, T, seed=1, precision="fp64", s0z=-1.0, tile_config=cfg, allow_unstable=True,
                    want_final_state=True)
        off = twa.run(p, B, dt, T, seed=1, precision="fp64", s0z=-1.0, tile_config=cfg, norm_tol=-1,
                      want_final_state=True)
        assert r.status == twa.TWA_EUNSTABLE and off.status == twa.TWA_OK
        dev = r.obs["max_norm_dev"]
        assert dev > 1e-2 and np.isfinite(r.obs["g2"]) and r.obs["nan_flag"] == 0
        assert np.array_equal(r.final_state, off.final_state) and r.obs["g2"] == off.obs["g2"]
        # the drift equals the largest | |s|^2 - |s0|^2 | of the returned state (|s0|^2 = 3),
        # reduced on the device in binary32
        norms = (r.final_state ** 2).sum(axis=0)
        assert abs(dev - np.max(np.abs(norms - 3.0))) < 1e-6 * dev
        assert twa.run(p, B, dt, T, seed=1, precision="fp64", s0z=-1.0, tile_config=cfg,
                       norm_tol=2 * dev).status == twa.TWA_OK
        s = twa.run(p, B, dt, T, seed=1, precision="fp64", s0z=-1.0, tile_config=cfg, integrator="sib")
        assert s.status == twa.TWA_OK and s.obs["max_norm_dev"] < 1e-10
    with pytest.raises(twa.TWAError) as e:
        twa.adjoint(p, B, dt, T, seed=1, precision="fp64", s0z=-1.0)
    assert e.value.code == twa.TWA_EUNSTABLE
    obs, g = twa.adjoint(p, B, dt, T, seed=1, precision="fp64", s0z=-1.0, allow_unstable=True)
    assert obs["max_norm_dev"] > 1e-2 and all(np.isfinite(v) for v in g.values())
    with pytest.raises(twa.TWAError) as e:
        twa.run_batch([(N, w, alpha, dt, 0), (40, w, alpha, dt, 1)], B, T, s0z=-1.0)
    assert e.value.code == twa.TWA_EUNSTABLE
