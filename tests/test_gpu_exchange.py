"""Coherent exchange (Omega_ij s+_i s-_j, i != j) on top of correlated decay
through the C ABI against the FP64 oracle: the third operand block
(s^y, -s^x) of the predictor and the second (D^y, -D^x) of the corrector, in
FP64 / FP32 / BF16 over ragged sizes and several tile configurations, with
Heun and the semi-implicit scheme; Omega = 0 against the model without it;
input checks."""
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


def _omega(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    O = scale * (A + A.T) / np.sqrt(n)
    np.fill_diagonal(O, 0.0)
    return O


def _oracle(N, w, alpha, G, O, B, dt, T, seed, **kw):
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=seed, decay=G, exchange=O,
                         **kw)
    return otwa.run(cfg, opump.build_pump(N, w, alpha))


@pytest.mark.parametrize("N,B,tile,integ", [(40, 50, -1, "heun"), (130, 70, 1, "heun"), (300, 40, 2, "heun"),
                                            (77, 33, 0, "sib"), (257, 20, 3, "heun")])
def test_fp64_matches_oracle(twa, N, B, tile, integ):
    w, alpha, dt, T, burn, seed = 2.0, 0.9, 2e-3, 160, 60, 5
    G = free_space_decay(N, 0.21, 0.8)
    O = _omega(N, N, 3.0)
    m = twa.build_model(opump.pump_matrix(N, w, alpha), G, O)
    r = twa.run(m, B, dt, T, seed=seed, precision="fp64", burnin=burn, tile_config=tile, integrator=integ,
                want_traj=True, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, G, O, B, dt, T, seed, burnin=burn, integrator=integ)
    for c in range(3):
        assert np.max(np.abs(r.final_state[c] - ref.final_state[c])) < 1e-11
    tg = ref.extra["traj_gen"]
    scale = np.abs(tg).max(axis=0) + 1e-300
    assert np.max(np.abs(r.traj_gen - tg) / scale) < 1e-10
    fin = odecay.finalize(tg)
    assert abs(r.obs["g2_gen"] - fin["g2"]) <= 1e-9 * abs(fin["g2"])


def test_exchange_changes_the_dynamics(twa):
    """The exchange is not a no-op at this strength: states move by far more
    than the parity tolerance relative to Omega = 0."""
    N, B, dt, T = 60, 16, 2e-3, 200
    G = random_psd(3, N)
    W = opump.pump_matrix(N, 1.5, 1.0)
    a = twa.run(twa.build_model(W, G, _omega(N, 7, 3.0)), B, dt, T, seed=1, precision="fp64", want_final_state=True, norm_tol=-1)
    b = twa.run(twa.build_model(W, G), B, dt, T, seed=1, precision="fp64", want_final_state=True, norm_tol=-1)
    assert np.max(np.abs(a.final_state - b.final_state)) > 1e-3


def test_zero_exchange_equals_the_decay_model(twa):
    N, B, dt, T = 100, 24, 2e-3, 150
    G = free_space_decay(N, 0.3, 1.0)
    W = opump.pump_matrix(N, 2.0, 0.8)
    a = twa.run(twa.build_model(W, G, np.zeros((N, N))), B, dt, T, seed=3, precision="fp64", want_final_state=True, norm_tol=-1)
    b = twa.run(twa.build_model(W, G), B, dt, T, seed=3, precision="fp64", want_final_state=True, norm_tol=-1)
    assert np.max(np.abs(a.final_state - b.final_state)) < 1e-12


def test_fp32_matches_oracle(twa):
    N, B, w, alpha, dt, T, burn, seed = 200, 64, 1.5, 1.1, 1e-3, 300, 150, 8
    G = free_space_decay(N, 0.12, 1.0)
    O = _omega(N, 11, 2.0)
    m = twa.build_model(opump.pump_matrix(N, w, alpha), G, O)
    r = twa.run(m, B, dt, T, seed=seed, precision="fp32", burnin=burn, want_traj=True, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, G, O, B, dt, T, seed, burnin=burn)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    assert (np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)).max() < 1e-5


@pytest.mark.parametrize("tile", [2, 7])
def test_bf16_matches_oracle_within_input_rounding(twa, tile):
    N, B, w, alpha, dt, T, burn, seed = 650, 130, 2.0, 1.0, 2e-4, 60, 30, 2
    G = free_space_decay(N, 0.3, 1.0)
    O = _omega(N, 13, 2.0)
    m = twa.build_model(opump.pump_matrix(N, w, alpha), G, O)
    r = twa.run(m, B, dt, T, seed=seed, precision="bf16", burnin=burn, tile_config=tile, want_final_state=True, norm_tol=-1)
    ref = _oracle(N, w, alpha, G, O, B, dt, T, seed, burnin=burn)
    g = r.final_state.transpose(1, 0, 2).reshape(B, -1)
    o = np.stack(ref.final_state).transpose(1, 0, 2).reshape(B, -1)
    assert (np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)).max() < 5e-3


def test_handle_and_errors(twa):
    N = 12
    W = opump.pump_matrix(N, 1.0, 1.0)
    G = free_space_decay(N, 0.2)
    O = _omega(N, 1)
    m = twa.build_model(W, G, O)
    assert np.array_equal(m.matrix("Omega"), O)
    bad = O.copy()
    bad[0, 0] = 0.5
    with pytest.raises(twa.TWAError) as e:
        twa.build_model(W, G, bad)
    assert e.value.code == -1
    asym = O.copy()
    asym[0, 1] += 0.2
    with pytest.raises(twa.TWAError):
        twa.build_model(W, G, asym)
    with pytest.raises(twa.TWAError):
        twa.run(m, 8, 1e-3, 20, precision="bf16x3", norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.run(m, 8, 1e-3, 20, precision="fp64", n_lags=4, norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.build_model(W, G).matrix("Omega")
