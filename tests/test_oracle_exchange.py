"""Pins of the oracle's coherent exchange (Omega_ij s+_i s-_j, i != j) added to
the correlated-decay model."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import decay, lindblad, pump, twa
from tests.inputs import free_space_decay, random_spins


def _omega(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    O = A + A.T
    np.fill_diagonal(O, 0.0)
    return O


def test_first_moments_at_t0_equal_the_heisenberg_rates_of_a_product_state():
    """For a product of pure single-spin states the exact rates d<sigma^a_i>/dt
    under H = sum_{i != j} Omega_ij sigma+_i sigma-_j factorise into the
    classical equations of motion at the Bloch vectors."""
    n = 3
    O = _omega(n, 2)
    rng = np.random.default_rng(5)
    kets = []
    for _ in range(n):
        v = rng.normal(size=2) + 1j * rng.normal(size=2)
        kets.append(v / np.linalg.norm(v))
    psi = kets[0]
    for k in kets[1:]:
        psi = np.kron(psi, k)
    sp, sm, sz = lindblad.operators(n)
    sx = [a + b for a, b in zip(sp, sm)]
    sy = [-1j * (a - b) for a, b in zip(sp, sm)]
    H = sum(O[i, j] * sp[i] @ sm[j] for i in range(n) for j in range(n) if i != j)

    def ev(op):
        return (psi.conj() @ op @ psi).real

    bloch = np.array([[ev(sx[i]), ev(sy[i]), ev(sz[i])] for i in range(n)])
    exact = np.array([[ev(1j * (H @ s[i] - s[i] @ H)) for s in (sx, sy, sz)] for i in range(n)])
    state = tuple(bloch[:, c][None, :] for c in range(3))
    dt = 1.0
    model = decay.Exchange(np.zeros((n, n)), O)
    zero = (np.zeros(1), np.zeros(1))
    inc = twa.increment(state, model, 0.0, dt, zero, (np.zeros((1, n)), np.zeros((1, n))))
    classical = np.stack([inc[0][0], inc[1][0], inc[2][0]], axis=1) / dt
    assert np.max(np.abs(classical - exact)) < 1e-12


def test_noiseless_exchange_conserves_energy_and_sz_at_second_order():
    n, B = 8, 3
    O = _omega(n, 3)
    s0 = tuple(random_spins(9, B, n))
    zeroW = np.zeros((n, n))

    def energy(st):
        x, y, _ = st
        return 0.25 * (np.einsum("ki,ij,kj->k", x, O, x) + np.einsum("ki,ij,kj->k", y, O, y))

    errs = []
    for dt in (2e-3, 1e-3):
        T = int(round(0.4 / dt))
        cfg = twa.RunConfig(n_spin=n, w=0.0, alpha=1.0, n_traj=B, dt=dt, n_steps=T, noise=False, init_state=s0,
                            burnin=0, gamma=0.0, exchange=O)
        res = twa.run(cfg, pump.Pump(n, 0.0, 1.0, zeroW, zeroW, np.zeros(n), np.eye(n), 0.0, 0.0))
        errs.append(np.max(np.abs(energy(res.final_state) - energy(s0))))
        assert np.max(np.abs(res.final_state[2].sum(1) - s0[2].sum(1))) < 1e-9
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 3.0   # at least second order (measured close to third)


def test_noiseless_full_model_vs_dop853():
    """Pump, correlated decay and coherent exchange together: second order
    against DOP853 of the field h^x = (1/2)(G s^x - W s^x) + (Omega s^y),
    h^y = (1/2)(G s^y - W s^y) - (Omega s^x)."""
    n, w, alpha = 6, 1.3, 0.8
    G = free_space_decay(n, 0.2, 1.0)
    O = _omega(n, 4) * 0.5
    W = pump.pump_matrix(n, w, alpha)
    s0 = tuple(random_spins(11, 1, n))
    T = 0.5

    def f(t, u):
        x, y, z = u.reshape(3, n)
        hx = 0.5 * G @ x - 0.5 * W @ x + O @ y
        hy = 0.5 * G @ y - 0.5 * W @ y - O @ x
        return np.concatenate([z * hx, z * hy, -(x * hx + y * hy)])

    ref = solve_ivp(f, (0, T), np.concatenate([a[0] for a in s0]), method="DOP853", rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for dt in (1e-2, 5e-3):
        cfg = twa.RunConfig(n_spin=n, w=w, alpha=alpha, n_traj=1, dt=dt, n_steps=int(round(T / dt)), noise=False,
                            init_state=s0, burnin=0, decay=G, exchange=O)
        fs = twa.run(cfg).final_state
        errs.append(np.max(np.abs(np.concatenate([a[0] for a in fs]) - ref)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_zero_exchange_is_the_decay_model():
    n, B = 7, 4
    G = free_space_decay(n, 0.3)
    base = dict(n_spin=n, w=1.5, alpha=1.0, n_traj=B, dt=1e-3, n_steps=60, seed=2, decay=G)
    a = twa.run(twa.RunConfig(**base))
    b = twa.run(twa.RunConfig(exchange=np.zeros((n, n)), **base))
    for u, v in zip(a.final_state, b.final_state):
        assert np.max(np.abs(u - v)) < 1e-15


def test_exchange_input_checks():
    with pytest.raises(ValueError):
        decay.Exchange(np.zeros((3, 3)), np.eye(3))
    O = _omega(3, 1)
    O[0, 1] += 1.0
    with pytest.raises(ValueError):
        decay.Exchange(np.zeros((3, 3)), O)
    with pytest.raises(NotImplementedError):
        twa.run(twa.RunConfig(n_spin=3, w=1.0, alpha=1.0, n_traj=2, dt=1e-3, n_steps=4, n_lags=2,
                              exchange=_omega(3, 1)))
