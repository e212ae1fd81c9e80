"""Pins of the correlated-decay oracle (the general-matrix extension of the
Perspectives; four-point function of SM Sec. S1 step 6)."""
import itertools
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import decay, lindblad, observables, philox, pump, twa
from tests.inputs import free_space_decay, random_psd, random_spins


def _site(op, i, n):
    out = np.array([[1.0 + 0j]])
    for k in range(n):
        out = np.kron(out, op if k == i else np.eye(2))
    return out


def _sym(ops):
    """Weyl (fully symmetrised) product of operators: the operator whose
    symmetric-order expectation the TWA average of the classical product is."""
    d = ops[0].shape[0]
    acc = np.zeros((d, d), dtype=np.complex128)
    for perm in itertools.permutations(range(len(ops))):
        m = np.eye(d, dtype=np.complex128)
        for j in perm:
            m = m @ ops[j]
        acc += m
    return acc / math.factorial(len(ops))


@pytest.mark.parametrize("n,which", [(2, "random"), (3, "random"), (3, "free")])
def test_estimator_is_an_exact_operator_identity(n, which):
    """With every TWA average replaced by the exact expectation of the Weyl-
    ordered operator (random mixed state, random PSD G), the intensity and
    four-point expressions of ``decay.derived`` equal the exact normal-ordered
    quantum values <sum G_ab s+_a s-_b> and sum G_ad G_bc <s+_a s+_b s-_c s-_d>
    (real parts: the TWA quantities are the Hermitian parts)."""
    G = random_psd(11 + n, n) if which == "random" else free_space_decay(n, 0.3, 0.7)
    sx = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    sy = np.array([[0, -1j], [1j, 0]])
    sz = np.diag([1.0 + 0j, -1.0])
    Z = [_site(sz, i, n) for i in range(n)]
    Pp = [(_site(sx, i, n) + 1j * _site(sy, i, n)) / 2 for i in range(n)]
    Pm = [(_site(sx, i, n) - 1j * _site(sy, i, n)) / 2 for i in range(n)]
    rng = np.random.default_rng(n)
    d = 2 ** n
    R = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    rho = R @ R.conj().T
    rho /= np.trace(rho)

    def ev(op):
        return np.trace(rho @ op).real

    r = range(n)
    E2 = sum(G[a, b] * ev(_sym([Pp[a], Pm[b]])) for a in r for b in r)
    E2E2 = sum(G[a, e] * G[b, c] * ev(_sym([Pp[a], Pm[e], Pp[b], Pm[c]])) for a in r for b in r for c in r for e in r)
    E2D = sum(G[a, a] * G[b, c] * ev(_sym([Pp[b], Pm[c], Z[a]])) for a in r for b in r for c in r)
    Q3 = sum(G[a, b] * G[b, c] * ev(_sym([Pp[a], Pm[c], Z[b]])) for a in r for b in r for c in r)
    Rv = sum(G[a, a] ** 2 * ev(Z[a]) for a in r)
    DD = sum(G[a, a] * G[b, b] * ev(_sym([Z[a], Z[b]])) for a in r for b in r)
    U = sum(G[a, b] * G[b, a] * ev(_sym([Z[a], Z[b]])) for a in r for b in r)
    V = sum(G[a, a] * G[a, b] * ev(_sym([Pp[a], Pm[b]])) for a in r for b in r)
    D = sum(G[a, a] * ev(Z[a]) for a in r)
    inten, g2 = decay.derived(np.array([E2, E2E2, E2D, Q3, Rv, DD, U, V, D]))
    exact_i = sum(G[a, b] * ev(Pp[a] @ Pm[b]) for a in r for b in r)
    exact_4 = sum(G[a, e] * G[b, c] * ev(Pp[a] @ Pp[b] @ Pm[c] @ Pm[e])
                  for a in r for b in r for c in r for e in r)
    assert abs(inten - exact_i) < 1e-12 * max(1.0, abs(exact_i))
    assert abs(g2 * inten * inten - exact_4) < 1e-11 * max(1.0, abs(exact_4))


def test_quantities_equal_brute_force_index_sums():
    """Each of the nine per-trajectory quantities against its defining sum
    over site indices, with s+- = (s^x +- i s^y)/2."""
    n, B = 4, 3
    G = random_psd(5, n)
    x, y, z = random_spins(7, B, n)
    q = decay.general_quantities((x, y, z), G)
    for k in range(B):
        sp = 0.5 * (x[k] + 1j * y[k])
        sm = 0.5 * (x[k] - 1j * y[k])
        r = range(n)
        E2 = sum(G[a, b] * sp[a] * sm[b] for a in r for b in r).real
        D = sum(G[a, a] * z[k, a] for a in r)
        Q3 = sum(G[a, b] * G[b, c] * sp[a] * sm[c] * z[k, b] for a in r for b in r for c in r).real
        Rv = sum(G[a, a] ** 2 * z[k, a] for a in r)
        U = sum(G[a, b] * G[b, a] * z[k, a] * z[k, b] for a in r for b in r)
        V = sum(G[a, a] * G[a, b] * sp[a] * sm[b] for a in r for b in r).real
        want = [E2, E2 * E2, E2 * D, Q3, Rv, D * D, U, V, D]
        assert np.allclose(q[k], want, rtol=1e-13, atol=1e-13)


def test_collective_limit_reduces_to_eq_s2():
    """G = Gamma0 * ones: intensity = Gamma0 <S+S-> of step 6 and g2 = Eq. (S2),
    state by state (for arbitrary classical states, not only sampled ones)."""
    n, B, g0 = 6, 50, 0.7
    s = random_spins(3, B, n)
    q = decay.general_quantities(tuple(s), g0 * np.ones((n, n)))
    m = twa.moments(tuple(s))
    for k in range(B):
        inten, g2 = decay.derived(q[k])
        _, spsm, g2c = observables.derived(m[k])
        assert abs(inten - g0 * spsm) < 1e-12 * max(1.0, abs(inten))
        assert abs(g2 - g2c) < 1e-10 * max(1.0, abs(g2c))


def _bits_states(n, s0z):
    for bits in itertools.product((-1.0, 1.0), repeat=2 * n):
        yield np.array(bits[:n]), np.array(bits[n:]), np.full(n, s0z)


@pytest.mark.parametrize("n,up,which", [(2, True, "random"), (2, False, "random"), (3, True, "free"),
                                        (3, False, "free")])
def test_sz_rate_at_t0_matches_lindblad_with_correlated_decay(n, up, which):
    """d<S^z>/dt at t = 0 of the correlated-decay step equals the exact rate of
    the master equation with correlated decay and correlated pump (expectation
    over the discrete initial law by enumeration and over the noise by an
    exact degree-3 cubature)."""
    G = random_psd(2, n) + 0.2 if which == "random" else free_space_decay(n, 0.2, 0.9)
    p = pump.build_pump(n, 1.3, 0.6)
    mp = decay.model_pump(p.W, G)
    ops = lindblad.operators(n)
    rho = lindblad.product_state(n, up)
    rate_q = lindblad.expect(lindblad.lindblad_rhs(rho, p.W, 0.0, ops, decay=G), sum(ops[2])).real
    expect = -2 * np.trace(G) if up else 2 * np.trace(p.W)
    assert abs(rate_q - expect) < 1e-12
    dt, d = 1e-7, 2 * n
    pts = []
    for k in range(d):
        for sg in (1.0, -1.0):
            v = np.zeros(d)
            v[k] = sg * np.sqrt(d)
            pts.append(v)
    tot, cnt = 0.0, 0
    zero = (np.zeros(1), np.zeros(1))
    for x, y, z in _bits_states(n, 1.0 if up else -1.0):
        st = (x[None, :], y[None, :], z[None, :])
        for v in pts:
            dchi = (np.sqrt(dt) * v[None, :n] @ mp.F.T, np.sqrt(dt) * v[None, n:] @ mp.F.T)
            new, _ = twa.heun_step(st, mp.W, 0.0, dt, zero, dchi)
            tot += (new[2] - st[2]).sum()
            cnt += 1
    assert abs(tot / cnt / dt - rate_q) < 1e-4 * abs(rate_q)


def test_noiseless_correlated_decay_vs_dop853():
    """No noise: the decay-mode Heun run converges at second order to the
    deterministic part of Eq. (S1) with the collective sum replaced by
    sum_j G_ij s_j (integrated independently with DOP853)."""
    n, w, alpha = 5, 1.5, 1.0
    G = free_space_decay(n, 0.25, 1.2)
    p = pump.build_pump(n, w, alpha)
    s0 = tuple(random_spins(4, 1, n))
    T = 0.5

    def f(t, u):
        x, y, z = u.reshape(3, n)
        hx = 0.5 * G @ x - 0.5 * p.W @ x
        hy = 0.5 * G @ y - 0.5 * p.W @ y
        return np.concatenate([z * hx, z * hy, -(x * hx + y * hy)])

    ref = solve_ivp(f, (0, T), np.concatenate([a[0] for a in s0]), method="DOP853", rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for dt in (1e-2, 5e-3):
        cfg = twa.RunConfig(n_spin=n, w=w, alpha=alpha, n_traj=1, dt=dt, n_steps=int(round(T / dt)), noise=False,
                            init_state=s0, burnin=0, decay=G)
        fs = twa.run(cfg, p).final_state
        errs.append(np.max(np.abs(np.concatenate([a[0] for a in fs]) - ref)))
    assert errs[0] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_noiseless_collective_limit_is_pathwise_identical():
    """G = Gamma * ones without noise reproduces the collective model's run."""
    n, B, gamma = 6, 4, 0.8
    s0 = tuple(random_spins(6, B, n))
    base = dict(n_spin=n, w=1.1, alpha=0.7, n_traj=B, dt=2e-3, n_steps=200, noise=False, init_state=s0, burnin=100)
    a = twa.run(twa.RunConfig(gamma=gamma, **base))
    b = twa.run(twa.RunConfig(decay=gamma * np.ones((n, n)), **base))
    for u, v in zip(a.final_state, b.final_state):
        assert np.max(np.abs(u - v)) < 1e-12
    # the general estimator reduces to Eq. (S2) along the trajectory
    mean = b.extra["traj_gen"].mean(0)
    inten, g2 = decay.derived(mean)
    _, spsm, g2c = observables.derived(a.traj_moments.mean(0))
    assert abs(inten - gamma * spsm) < 1e-10 * abs(inten)
    assert abs(g2 - g2c) < 1e-9 * abs(g2c)


def test_noise_covariance_is_pump_plus_decay():
    """The per-step noise of the decay mode has covariance (W + G) dt per
    component, independent between x and y (sample covariance over 40000
    trajectories within 6 standard errors)."""
    n, B, dt = 5, 40000, 1e-2
    G = free_space_decay(n, 0.15, 1.0)
    p = pump.build_pump(n, 0.8, 1.3)
    mp = decay.model_pump(p.W, G)
    cfg = twa.RunConfig(n_spin=n, w=0.8, alpha=1.3, n_traj=B, dt=dt, n_steps=1, seed=12, gamma=0.0)
    _, dchi = twa.noise_increments(cfg, mp, 0)
    target = (p.W + G) * dt
    for c in (0, 1):
        emp = dchi[c].T @ dchi[c] / B
        se = np.sqrt((np.outer(np.diag(target), np.diag(target)) + target ** 2) / B)
        assert np.max(np.abs(emp - target) / se) < 6.0
    cross = dchi[0].T @ dchi[1] / B
    se = np.sqrt(np.outer(np.diag(target), np.diag(target)) / B)
    assert np.max(np.abs(cross) / se) < 6.0


def test_model_matrices():
    n = 7
    G = free_space_decay(n, 0.1)
    W = pump.pump_matrix(n, 1.0, 0.5)
    mp = decay.model_pump(W, G)
    assert np.allclose(mp.W, W - G, atol=0)
    assert np.allclose(mp.F @ mp.F, W + G, atol=1e-12)
    assert np.allclose(mp.F, mp.F.T, atol=0)
    assert np.min(np.linalg.eigvalsh(mp.F)) > -1e-12


def test_finalize_jackknife_and_lag_rejection():
    B, n = 64, 4
    G = random_psd(1, n)
    q = decay.general_quantities(tuple(random_spins(2, B, n)), G)
    out = decay.finalize(q)
    inten, g2 = decay.derived(q.mean(0))
    assert out["I"] == pytest.approx(inten, rel=1e-14) and out["g2"] == pytest.approx(g2, rel=1e-14)
    assert out["I_se"] > 0 and out["g2_se"] > 0
    with pytest.raises(NotImplementedError):
        twa.run(twa.RunConfig(n_spin=n, w=1.0, alpha=1.0, n_traj=2, dt=1e-3, n_steps=4, n_lags=2, decay=G))
