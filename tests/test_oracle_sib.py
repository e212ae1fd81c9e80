"""Pins of the oracle's semi-implicit midpoint integrator (the scheme the paper
cites for its spin-length-preserving integration, Mentink et al. 2010): each
stage is a rotation of every spin, so the length is kept exactly; the scheme
is second order; and its stationary statistics match the exact law."""
import numpy as np
from scipy.integrate import solve_ivp

from oracle import closed_forms, observables, pump, twa


def _rodrigues(s, k, phi):
    """Rotation of the vectors s (..., 3) about the unit axes k by the angles phi."""
    c, sn = np.cos(phi)[..., None], np.sin(phi)[..., None]
    return s * c + np.cross(k, s) * sn + k * np.sum(k * s, axis=-1, keepdims=True) * (1 - c)


def test_midpoint_stage_is_the_rotation_about_minus_b():
    """ds = s x b = (-b) x s: the midpoint rule with b frozen is the rotation about
    -b/|b| by 2 arctan(|b|/2) (Cayley transform of the rotation generator)."""
    rng = np.random.default_rng(1)
    B, n = 4, 5
    st = tuple(rng.standard_normal((B, n)) for _ in range(3))
    hx, hy = 0.7 * rng.standard_normal((B, n)), 0.7 * rng.standard_normal((B, n))
    out = np.stack(twa.midpoint_rotation(st, hx, hy), axis=-1)
    b = np.stack([hy, -hx, np.zeros_like(hx)], axis=-1)
    nb = np.linalg.norm(b, axis=-1)
    ref = _rodrigues(np.stack(st, axis=-1), -b / nb[..., None], 2 * np.arctan(nb / 2))
    assert np.max(np.abs(out - ref)) < 1e-13


def test_sib_keeps_spin_length_with_noise():
    n, B, dt, T = 6, 16, 5e-3, 200
    kw = dict(n_spin=n, w=2.0, alpha=1.0, n_traj=B, dt=dt, n_steps=T, seed=4, burnin=0)
    sib = twa.run(twa.RunConfig(integrator="sib", **kw))
    heun = twa.run(twa.RunConfig(**kw))
    assert sib.max_norm_dev < 1e-12
    assert heun.max_norm_dev > 1e-4     # Heun's first-order length drift, for contrast


def test_sib_noiseless_collective_decay_closed_form_second_order():
    """alpha = 0, identical spins, no noise: s^z(t) = -r tanh(kappa r (t - t_D))."""
    n, gamma, w = 6, 1.0, 0.4
    z0, x0 = 0.9, np.sqrt(3.0 - 0.81)
    r, T = np.sqrt(3.0), 0.4
    errs = []
    for dt in (2e-3, 1e-3):
        init = (np.full((1, n), x0), np.zeros((1, n)), np.full((1, n), z0))
        cfg = twa.RunConfig(n_spin=n, w=w, alpha=0.0, n_traj=1, dt=dt, n_steps=int(round(T / dt)),
                            gamma=gamma, noise=False, init_state=init, burnin=0, integrator="sib")
        zT = twa.run(cfg).final_state[2][0, 0]
        errs.append(abs(zT - closed_forms.noiseless_collective_z(T, n, gamma, w, r, z0)))
    assert errs[0] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_sib_noiseless_correlated_pump_vs_dop853():
    n, gamma, w, alpha, T = 5, 1.0, 2.0, 1.0, 0.5
    p = pump.build_pump(n, w, alpha)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, n))
    v *= np.sqrt(3.0) / np.linalg.norm(v, axis=0)
    s0 = tuple(v[c][None, :] for c in range(3))

    def f(t, u):
        x, y, z = u.reshape(3, n)
        hx = 0.5 * gamma * x.sum() - 0.5 * p.W @ x
        hy = 0.5 * gamma * y.sum() - 0.5 * p.W @ y
        return np.concatenate([z * hx, z * hy, -(x * hx + y * hy)])

    ref = solve_ivp(f, (0, T), v.reshape(-1), method="DOP853", rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for dt in (1e-2, 5e-3):
        cfg = twa.RunConfig(n_spin=n, w=w, alpha=alpha, n_traj=1, dt=dt, n_steps=int(round(T / dt)),
                            gamma=gamma, noise=False, init_state=s0, burnin=0, integrator="sib")
        fs = twa.run(cfg, p).final_state
        errs.append(np.max(np.abs(np.concatenate([a[0] for a in fs]) - ref)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_sib_alpha0_stationary_law_monte_carlo():
    """alpha = 0, w = Gamma/2, N = 10: the exact stationary law of the rigidly
    rotating collective spin (-7.940, 7.940, 1.519), within 4 standard errors
    plus 1.5 % (1024 trajectories, 2000 window steps at dt = 1e-3)."""
    n, gamma, w = 10, 1.0, 0.5
    ez, es, eg = observables.derived(closed_forms.stationary_alpha0(n, gamma, w))
    cfg = twa.RunConfig(n_spin=n, w=w, alpha=0.0, n_traj=1024, dt=1e-3, n_steps=3000, seed=2, burnin=1000,
                        integrator="sib")
    m = observables.finalize(twa.run(cfg).traj_moments)
    for key, ref in (("Sz", ez), ("SpSm", es), ("g2", eg)):
        tol = 4 * m[key + "_se"] + 0.015 * abs(ref)
        assert abs(m[key] - ref) < tol, (key, m[key], ref, m[key + "_se"])
