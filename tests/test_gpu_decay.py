"""Correlated decay through the C ABI against the FP64 oracle: the model
handle's matrices, the step (drift W - G, noise factor sqrt(W + G), no
collective terms) and the correlated-emission estimator (nine quantities per
trajectory, intensity and g2), in FP64 / FP32 / BF16 over ragged sizes and
several tile configurations; the collective limit against the run's own
collective moments at a larger size; sampled trajectories at N = 2048; error
paths."""
import numpy as np
import pytest

from oracle import decay as odecay
from oracle import pump as opump
from oracle import twa as otwa
from tests.inputs import free_space_decay, random_psd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def _oracle(N, w, alpha, G, B, dt, T, seed, **kw):
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=seed, decay=G, **kw)
    return otwa.run(cfg, opump.build_pump(N, w, alpha))


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def test_model_handle_matrices(twa):
    N = 37
    W = opump.pump_matrix(N, 1.7, 0.8)
    G = free_space_decay(N, 0.3, 1.1)
    m = twa.build_model(W, G)
    assert m.has_decay
    assert np.max(np.abs(m.matrix("W") - (W - G))) < 1e-15
    assert np.max(np.abs(m.matrix("G") - G)) == 0.0
    F = m.matrix("F")
    assert np.max(np.abs(F @ F - (W + G))) < 1e-12
    lam = np.linalg.eigvalsh(W + G)
    assert abs(m.lam_max - lam[-1]) < 1e-12 * lam[-1]
    assert abs(m.lam_min - lam[0]) < 1e-10 * lam[-1]


@pytest.mark.parametrize("N,B,tile,which,integ", [
    (40, 50, -1, "free", "heun"),      # automatic tile (16 x 32)
    (130, 70, 1, "random", "heun"),    # ragged N and B, 64 x 64 tiles
    (300, 40, 2, "free", "heun"),      # 128 x 128 tiles, one column tile
    (77, 33, 0, "free", "sib"),        # semi-implicit integrator
])
def test_fp64_matches_oracle(twa, N, B, tile, which, integ):
    w, alpha, dt, T, burn, seed = 2.0, 0.9, 2e-3, 160, 60, 5
    G = free_space_decay(N, 0.21, 0.8) if which == "free" else random_psd(9, N, rank=N // 3)
    m = twa.build_model(opump.pump_matrix(N, w, alpha), G)
    r = twa.run(m, B, dt, T, seed=seed, precision="fp64", burnin=burn, tile_config=tile, integrator=integ,
                want_traj=True, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, G, B, dt, T, seed, burnin=burn, integrator=integ)
    assert r.obs["tile_config"] != 99
    for c in range(3):
        assert np.max(np.abs(r.final_state[c] - ref.final_state[c])) < 1e-11
    assert _rel(r.traj_moments, ref.traj_moments) < 1e-10
    tg = ref.extra["traj_gen"]
    scale = np.abs(tg).max(axis=0) + 1e-300
    assert np.max(np.abs(r.traj_gen - tg) / scale) < 1e-10
    fin = odecay.finalize(tg)
    for gk, ok in (("I_gen", "I"), ("g2_gen", "g2"), ("I_gen_se", "I_se"), ("g2_gen_se", "g2_se")):
        assert abs(r.obs[gk] - fin[ok]) <= 1e-9 * max(1.0, abs(fin[ok])), gk


def test_fp32_matches_oracle(twa):
    N, B, w, alpha, dt, T, burn, seed = 200, 64, 1.5, 1.1, 1e-3, 300, 150, 8
    G = free_space_decay(N, 0.12, 1.0)
    m = twa.build_model(opump.pump_matrix(N, w, alpha), G)
    r = twa.run(m, B, dt, T, seed=seed, precision="fp32", burnin=burn, want_traj=True, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, G, B, dt, T, seed, burnin=burn)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    assert (np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)).max() < 1e-5
    tg = ref.extra["traj_gen"]
    scale = np.abs(tg).max(axis=0)
    assert np.max(np.abs(r.traj_gen - tg) / scale) < 2e-5
    fin = odecay.finalize(tg)
    assert abs(r.obs["I_gen"] - fin["I"]) < 2e-5 * abs(fin["I"])
    assert abs(r.obs["g2_gen"] - fin["g2"]) < 2e-5 * abs(fin["g2"])


@pytest.mark.parametrize("tile", [2, 7])
def test_bf16_matches_oracle_within_input_rounding(twa, tile):
    """BF16 contraction inputs (state and matrices rounded to 8 significant
    bits, FP32 accumulation): per-trajectory estimator quantities within the
    rounding-error band of a short run."""
    N, B, w, alpha, dt, T, burn, seed = 650, 130, 2.0, 1.0, 2e-4, 60, 30, 2
    G = free_space_decay(N, 0.3, 1.0)
    m = twa.build_model(opump.pump_matrix(N, w, alpha), G)
    r = twa.run(m, B, dt, T, seed=seed, precision="bf16", burnin=burn, tile_config=tile, want_traj=True,
                want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, G, B, dt, T, seed, burnin=burn)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    assert (np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)).max() < 5e-3
    tg = ref.extra["traj_gen"]
    scale = np.abs(tg).max(axis=0)
    assert np.max(np.abs(r.traj_gen - tg) / scale) < 2e-2
    fin = odecay.finalize(tg)
    assert abs(r.obs["I_gen"] - fin["I"]) < 1e-2 * abs(fin["I"])


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-5), ("fp64", 1e-11)])
def test_collective_limit_equals_the_runs_own_eq_s2(twa, precision, tol):
    """G = gamma * ones: the correlated-emission estimator of every observed
    state equals gamma * <S+S-> and Eq. (S2) of the same trajectories."""
    N, B, gamma = 1000 if precision == "fp32" else 260, 96, 0.7
    W = opump.pump_matrix(N, 0.5, 0.6)
    m = twa.build_model(W, gamma * np.ones((N, N)))
    r = twa.run(m, B, 0.02 / N, 200, seed=4, precision=precision, want_traj=True, norm_tol=-1)
    inten = r.traj_gen[:, 0] + 0.5 * r.traj_gen[:, 8]
    spsm = r.traj_moments[:, 0] + 0.5 * r.traj_moments[:, 3]
    assert np.max(np.abs(inten - gamma * spsm)) < tol * np.max(np.abs(gamma * spsm))
    assert abs(r.obs["I_gen"] - gamma * r.obs["SpSm"]) < tol * abs(gamma * r.obs["SpSm"])
    assert abs(r.obs["g2_gen"] - r.obs["g2"]) < 50 * tol * abs(r.obs["g2"])


def test_large_n_sampled_trajectories(twa):
    """N = 2048, 256 trajectories, FP32: three trajectories re-integrated by the
    oracle alone (trajectories are independent)."""
    N, B, w, alpha, dt, T, burn, seed = 2048, 256, 3.0, 0.7, 1e-5, 12, 6, 21
    G = free_space_decay(N, 0.05, 1.0)
    m = twa.build_model(opump.pump_matrix(N, w, alpha), G)
    r = twa.run(m, B, dt, T, seed=seed, precision="fp32", burnin=burn, want_traj=True, want_final_state=True, norm_tol=-1)
    idx = np.array([0, 131, 255])
    ref = _oracle(N, w, alpha, G, 3, dt, T, seed, burnin=burn, traj=idx)
    for j, k in enumerate(idx):
        got = r.final_state[:, k, :]
        want = np.stack([ref.final_state[c][j] for c in range(3)])
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-5
        tg = ref.extra["traj_gen"][j]
        assert np.max(np.abs(r.traj_gen[k] - tg) / (np.abs(tg) + 1e-3 * np.abs(tg).max())) < 1e-4


def test_errors(twa):
    N = 12
    W = opump.pump_matrix(N, 1.0, 1.0)
    m = twa.build_model(W, free_space_decay(N, 0.2))
    with pytest.raises(twa.TWAError):
        twa.run(m, 8, 1e-3, 20, n_lags=4, precision="fp64", norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.adjoint(m, 8, 1e-3, 20, norm_tol=-1)
    bad = free_space_decay(N, 0.2)
    bad[0, 0] = -1.0
    with pytest.raises(twa.TWAError) as e:
        twa.build_model(W, bad)
    assert e.value.code == -4
    asym = free_space_decay(N, 0.2)
    asym[0, 1] += 0.1
    with pytest.raises(twa.TWAError) as e:
        twa.build_model(W, asym)
    assert e.value.code == -1
    # without a model handle the decay outputs are NaN
    r = twa.run(twa.build_pump(N, 1.0, 1.0), 8, 1e-3, 20, precision="fp64", norm_tol=-1)
    assert np.isnan(r.obs["I_gen"]) and np.isnan(r.obs["g2_gen"])
