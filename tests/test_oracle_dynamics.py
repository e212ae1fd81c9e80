"""Pins of the oracle's equations of motion and Heun integrator."""
import itertools

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import closed_forms, lindblad, observables, pump, twa


def _random_state(rng, B, n):
    v = rng.normal(size=(3, B, n))
    v *= np.sqrt(3.0) / np.linalg.norm(v, axis=0)
    return tuple(v)


def test_increment_orthogonal_to_spin():
    """Eq. (S1) is s x b: the increment is orthogonal to s (length preserved)."""
    rng = np.random.default_rng(0)
    p = pump.build_pump(9, 1.3, 0.7)
    s = _random_state(rng, 6, 9)
    dxi = (rng.normal(size=6), rng.normal(size=6))
    dchi = (rng.normal(size=(6, 9)), rng.normal(size=(6, 9)))
    d = twa.increment(s, p.W, 1.0, 1e-2, dxi, dchi)
    dot = s[0] * d[0] + s[1] * d[1] + s[2] * d[2]
    assert np.max(np.abs(dot)) < 1e-14


def test_heun_norm_error_is_second_order_per_step():
    rng = np.random.default_rng(1)
    p = pump.build_pump(8, 2.0, 1.0)
    s = _random_state(rng, 4, 8)
    errs = []
    for dt in (1e-3, 5e-4):
        dxi = (np.sqrt(dt) * rng.normal(size=4) * 0, np.zeros(4))
        dchi = (np.zeros((4, 8)), np.zeros((4, 8)))
        new, _ = twa.heun_step(s, p.W, 1.0, dt, dxi, dchi)
        errs.append(np.max(np.abs(sum(a * a for a in new) - 3.0)))
    assert errs[1] < errs[0] / 3.0


def _bits_states(n, s0z):
    for bits in itertools.product((-1.0, 1.0), repeat=2 * n):
        x = np.array(bits[:n])
        y = np.array(bits[n:])
        yield x, y, np.full(n, s0z)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_initial_moments_exact_enumeration(n):
    """Discrete sampling: <s^a> = 0, <(s^a)^2> = 1 and <S+S-> equals the quantum
    value N (all excited) / 0 (all ground) exactly."""
    for s0z, expect in ((1.0, n), (-1.0, 0.0)):
        states = list(_bits_states(n, s0z))
        X = np.array([s[0] for s in states])
        Y = np.array([s[1] for s in states])
        Z = np.array([s[2] for s in states])
        assert np.allclose(X.mean(0), 0) and np.allclose((X * X).mean(0), 1)
        assert np.allclose((X * Y).mean(0), 0)
        m = twa.moments((X, Y, Z)).mean(0)
        _, spsm, _ = observables.derived(m)
        assert abs(spsm - expect) < 1e-12


def test_sampled_initial_state():
    x, y, z = twa.initial_state(seed=0, n_traj=4000, n_spin=6, s0z=1.0)
    m = observables.finalize(twa.moments((x, y, z)))
    assert abs(m["SpSm"] - 6.0) < 4 * m["SpSm_se"]
    assert np.all(z == 1.0)


@pytest.mark.parametrize("n,up", [(2, True), (2, False), (3, True), (3, False)])
def test_sz_rate_at_t0_matches_lindblad(n, up):
    """d<S^z>/dt at t = 0 from the TWA step equals the exact Lindblad rate of
    Eq. (1) for a correlated pump (expectation over the discrete initial law by
    enumeration and over the noise by a degree-3 exact cubature)."""
    gamma = 0.8
    p = pump.build_pump(n, 1.3, 0.6)
    # exact quantum rate
    ops = lindblad.operators(n)
    rho = lindblad.product_state(n, up)
    drho = lindblad.lindblad_rhs(rho, p.W, gamma, ops)
    Sz = sum(ops[2])
    rate_q = lindblad.expect(drho, Sz).real
    # TWA: E[Delta S^z] / dt for a tiny dt
    dt = 1e-7
    d = 2 + 2 * n
    pts = []
    for k in range(d):
        for sgn in (1.0, -1.0):
            v = np.zeros(d)
            v[k] = sgn * np.sqrt(d)
            pts.append(v)
    tot = 0.0
    cnt = 0
    for x, y, z in _bits_states(n, 1.0 if up else -1.0):
        st = (x[None, :], y[None, :], z[None, :])
        for v in pts:
            g = (np.array([v[0]]), np.array([v[1]]))
            zx, zy = v[2:2 + n][None, :], v[2 + n:][None, :]
            dxi = (np.sqrt(gamma * dt) * g[0], np.sqrt(gamma * dt) * g[1])
            dchi = (np.sqrt(dt) * zx @ p.F.T, np.sqrt(dt) * zy @ p.F.T)
            new, _ = twa.heun_step(st, p.W, gamma, dt, dxi, dchi)
            tot += (new[2] - st[2]).sum()
            cnt += 1
    rate_twa = tot / cnt / dt
    expect = -2 * gamma * n if up else 2 * np.trace(p.W)
    assert abs(rate_q - expect) < 1e-12
    assert abs(rate_twa - rate_q) < 1e-4 * abs(rate_q)


def test_noiseless_collective_decay_closed_form_second_order():
    """alpha = 0, identical spins, no noise: s^z(t) = -r tanh(kappa r (t - t_D))."""
    n, gamma, w = 6, 1.0, 0.4
    z0, x0 = 0.9, np.sqrt(3.0 - 0.81)
    r = np.sqrt(3.0)
    T = 0.4
    errs = []
    for dt in (2e-3, 1e-3):
        steps = int(round(T / dt))
        init = (np.full((1, n), x0), np.zeros((1, n)), np.full((1, n), z0))
        cfg = twa.RunConfig(n_spin=n, w=w, alpha=0.0, n_traj=1, dt=dt, n_steps=steps,
                            gamma=gamma, noise=False, init_state=init, burnin=0)
        res = twa.run(cfg)
        zT = res.final_state[2][0, 0]
        errs.append(abs(zT - closed_forms.noiseless_collective_z(T, n, gamma, w, r, z0)))
    assert errs[0] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_noiseless_correlated_pump_vs_dop853():
    n, gamma, w, alpha = 5, 1.0, 2.0, 1.0
    p = pump.build_pump(n, w, alpha)
    rng = np.random.default_rng(3)
    s0 = _random_state(rng, 1, n)
    T = 0.5

    def f(t, u):
        x, y, z = u.reshape(3, n)
        hx = 0.5 * gamma * x.sum() - 0.5 * p.W @ x
        hy = 0.5 * gamma * y.sum() - 0.5 * p.W @ y
        return np.concatenate([z * hx, z * hy, -(x * hx + y * hy)])

    ref = solve_ivp(f, (0, T), np.concatenate([a[0] for a in s0]), method="DOP853",
                    rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for dt in (1e-2, 5e-3):
        cfg = twa.RunConfig(n_spin=n, w=w, alpha=alpha, n_traj=1, dt=dt, n_steps=int(round(T / dt)),
                            gamma=gamma, noise=False, init_state=s0, burnin=0)
        fs = twa.run(cfg, p).final_state
        errs.append(np.max(np.abs(np.concatenate([a[0] for a in fs]) - ref)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_local_limit_matches_diagonal_implementation():
    """alpha = 60: the general path equals an implementation with w_ij = w delta_ij."""
    n, B, w, dt = 7, 16, 1.5, 1e-3
    cfg = twa.RunConfig(n_spin=n, w=w, alpha=60.0, n_traj=B, dt=dt, n_steps=50, seed=4, burnin=0)
    res = twa.run(cfg)
    from oracle import philox
    x, y, z = twa.initial_state(4, B, n, 1.0)
    for step in range(50):
        gx, gy = philox.collective_noise(4, step, B)
        zx, zy = philox.pump_noise(4, step, B, n)

        def incr(x, y, z):
            hx = (0.5 * x.sum(1)[:, None] - 0.5 * w * x) * dt + np.sqrt(dt) * gx[:, None] - np.sqrt(w * dt) * zx
            hy = (0.5 * y.sum(1)[:, None] - 0.5 * w * y) * dt + np.sqrt(dt) * gy[:, None] - np.sqrt(w * dt) * zy
            return z * hx, z * hy, -(x * hx + y * hy)

        a = incr(x, y, z)
        b = incr(x + a[0], y + a[1], z + a[2])
        x, y, z = x + 0.5 * (a[0] + b[0]), y + 0.5 * (a[1] + b[1]), z + 0.5 * (a[2] + b[2])
    for u, v in zip(res.final_state, (x, y, z)):
        assert np.max(np.abs(u - v)) < 1e-12


def test_determinism():
    cfg = twa.RunConfig(n_spin=6, w=1.0, alpha=1.0, n_traj=8, dt=1e-3, n_steps=40, seed=9, n_lags=4)
    a, b = twa.run(cfg), twa.run(cfg)
    assert np.array_equal(a.traj_moments, b.traj_moments)
    assert np.array_equal(a.corr_blocks, b.corr_blocks)


def test_blas_thread_count_changes_only_rounding():
    """At a fixed BLAS thread count the oracle is bitwise reproducible; the
    matrix products are BLAS calls whose summation split depends on the
    thread count, so 1 and 4 threads agree to rounding (measured 2e-15 on
    unit spins), not bit for bit."""
    from threadpoolctl import threadpool_limits
    cfg = twa.RunConfig(n_spin=300, w=2.0, alpha=1.0, n_traj=64, dt=1e-4, n_steps=30, seed=2)
    with threadpool_limits(limits=1):
        a, a2 = twa.run(cfg), twa.run(cfg)
    with threadpool_limits(limits=4):
        b = twa.run(cfg)
    for u, u2, v in zip(a.final_state, a2.final_state, b.final_state):
        assert np.array_equal(u, u2)
        assert np.max(np.abs(u - v)) < 1e-12
    assert np.max(np.abs(a.traj_moments - b.traj_moments) / (np.abs(a.traj_moments) + 1e-300)) < 1e-12


def test_trajectory_subset_equals_rows_of_full_ensemble():
    """Trajectories are independent (their noise counters carry the trajectory
    index), so integrating a subset reproduces those rows of the full run."""
    n, B, T = 7, 9, 25
    full = twa.run(twa.RunConfig(n_spin=n, w=1.7, alpha=0.8, n_traj=B, dt=2e-3, n_steps=T, seed=3, s0z=-1.0))
    idx = np.array([8, 0, 5])
    sub = twa.run(twa.RunConfig(n_spin=n, w=1.7, alpha=0.8, n_traj=3, dt=2e-3, n_steps=T, seed=3, s0z=-1.0,
                                traj=idx))
    for c in range(3):
        assert np.array_equal(sub.final_state[c], full.final_state[c][idx])
    assert np.array_equal(sub.traj_moments, full.traj_moments[idx])
