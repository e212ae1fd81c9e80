"""Pins of the oracle's pathwise parameter derivatives."""
import numpy as np

from oracle import grad, twa


def test_pathwise_gradient_matches_central_differences():
    cfg = twa.RunConfig(n_spin=6, w=2.0, alpha=1.0, n_traj=24, dt=2e-3, n_steps=300, seed=7, burnin=150)
    g = grad.pathwise_gradients(cfg)
    fd = grad.fd_gradients(cfg, h=1e-4)
    for key, v in fd.items():
        scale = max(abs(v), 1e-3)
        assert abs(g[key] - v) < 1e-5 * scale + 1e-8, (key, g[key], v)


def test_pathwise_gradient_alpha0_w_direction():
    # at alpha = 0 the w-derivative is still well defined (rank-one pump)
    cfg = twa.RunConfig(n_spin=4, w=0.7, alpha=0.0, n_traj=16, dt=2e-3, n_steps=120, seed=1, burnin=60)
    g = grad.pathwise_gradients(cfg)
    fd = grad.fd_gradients(cfg, h=1e-4, params=("w",))
    for name in ("Sz", "SpSm", "g2"):
        key = "d_%s_dw" % name
        assert abs(g[key] - fd[key]) < 1e-5 * max(abs(fd[key]), 1e-3) + 1e-8


def _rand_state(rng, B, n, scale=1.0):
    return tuple(scale * rng.standard_normal((B, n)) for _ in range(3))


def _dot(a, b):
    return float(sum(np.sum(x * y) for x, y in zip(a, b)))


def test_heun_vjp_is_the_transpose_of_the_tangent_step():
    """Dot-product test of the reverse-mode Heun step against the tangent-linear
    step (<u, J v> = <J^T u, v>, FP64 to 1e-12).  A random non-symmetric
    matrix stands in for W so that a transposed product in either mode fails;
    nonzero Gamma and noise keep every term of the field in play."""
    rng = np.random.default_rng(11)
    for B, n, gamma, dt in ((3, 5, 1.0, 1e-2), (4, 9, 0.7, 5e-2), (2, 16, 2.0, 2e-3)):
        W = rng.standard_normal((n, n))
        state = _rand_state(rng, B, n)
        dxi = tuple(0.3 * rng.standard_normal(B) for _ in range(2))
        dchi = tuple(0.3 * rng.standard_normal((B, n)) for _ in range(2))
        for _ in range(4):
            v, u = _rand_state(rng, B, n), _rand_state(rng, B, n)
            Jv = twa.heun_step_tangent(state, v, W, gamma, dt, dxi, dchi)
            JTu = grad.heun_step_vjp(state, u, W, gamma, dt, dxi, dchi)
            a, b = _dot(u, Jv), _dot(JTu, v)
            assert abs(a - b) <= 1e-12 * max(abs(a), 1.0), (a, b)


def test_reverse_sweep_over_many_steps_matches_tangent_propagation():
    """The same identity through 25 Heun steps of a real run (Eq. (2) pump,
    Philox noise): the reverse sweep over stored states against the tangent
    propagated forward."""
    from oracle import philox, pump
    cfg = twa.RunConfig(n_spin=12, w=3.0, alpha=0.9, n_traj=6, dt=4e-3, n_steps=25, seed=4)
    p = pump.build_pump(cfg.n_spin, cfg.w, cfg.alpha)
    rng = np.random.default_rng(2)
    state = twa.initial_state(cfg.seed, cfg.n_traj, cfg.n_spin)
    v = _rand_state(rng, cfg.n_traj, cfg.n_spin)
    u = _rand_state(rng, cfg.n_traj, cfg.n_spin)
    states, noises, t = [], [], v
    for n in range(cfg.n_steps):
        dxi, dchi = twa.noise_increments(cfg, p, n)
        states.append(state)
        noises.append((dxi, dchi))
        t = twa.heun_step_tangent(state, t, p.W, cfg.gamma, cfg.dt, dxi, dchi)
        state = twa.heun_step(state, p.W, cfg.gamma, cfg.dt, dxi, dchi)[0]
    lam = u
    for n in reversed(range(cfg.n_steps)):
        lam = grad.heun_step_vjp(states[n], lam, p.W, cfg.gamma, cfg.dt, *noises[n])
    a, b = _dot(u, t), _dot(lam, v)
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0), (a, b)
