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
