"""Pins of the pump matrix, its channel decomposition and the PSD factor."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import pump


@pytest.mark.parametrize("n,w,alpha", [(7, 1.3, 0.0), (33, 2.0, 0.5), (64, 0.7, 1.0), (50, 4.0, 2.7)])
def test_factor_squares_to_w(n, w, alpha):
    p = pump.build_pump(n, w, alpha)
    assert np.allclose(p.F, p.F.T, atol=0)
    assert np.max(np.abs(p.F @ p.F - p.W)) <= 1e-12 * np.max(np.abs(p.W)) * n
    assert np.min(np.linalg.eigvalsh(p.F)) > -1e-10 * p.lam_max ** 0.5
    # independent route: scipy's matrix square root of the same W
    if alpha > 0:
        assert np.allclose(np.real(sla.sqrtm(p.W)), p.F, atol=1e-9)


def test_matrix_entries_eq2():
    W = pump.pump_matrix(5, 3.0, 1.5)
    assert W[0, 0] == 3.0 and W[4, 4] == 3.0
    assert np.isclose(W[0, 3], 3.0 / 4 ** 1.5) and np.isclose(W[3, 0], W[0, 3])
    assert np.isclose(W[1, 2], 3.0 / 2 ** 1.5)


def test_collective_limit_rank_one():
    n, w = 40, 0.8
    p = pump.build_pump(n, w, 0.0)
    assert np.isclose(p.lam_max, w * n, rtol=1e-13)
    assert np.all(np.abs(p.lam[:-1]) < 1e-12 * w * n)
    assert np.allclose(p.F, np.sqrt(w / n) * np.ones((n, n)), atol=1e-13)


def test_local_limit():
    p = pump.build_pump(30, 2.5, 60.0)
    assert np.allclose(p.W, 2.5 * np.eye(30), rtol=0, atol=2.5 * 2.0 ** -59)
    assert np.allclose(p.F, np.sqrt(2.5) * np.eye(30), atol=1e-15)


def test_pd_for_positive_alpha_grid():
    for alpha in np.linspace(0.25, 3.0, 12):
        p = pump.build_pump(200, 1.0, alpha)
        assert p.lam_min > 0


def test_dirichlet_eta_special_values():
    assert np.isclose(pump.dirichlet_eta(1.0), np.log(2.0), rtol=1e-9)
    assert np.isclose(pump.dirichlet_eta(2.0), np.pi ** 2 / 12.0, rtol=1e-9)


@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.0])
def test_lambda_min_eta_law(alpha):
    """Smallest channel rate -> w (2 eta(alpha) - 1) (text after Eq. (3))."""
    p = pump.build_pump(1000, 1.0, alpha)
    est = pump.lam_min_estimate(1.0, alpha)
    assert abs(p.lam_min - est) / est < 1e-3


def test_lambda_max_scaling_eq3():
    """Eq. (3): w N^(1-alpha) for alpha < 1, w log N at alpha = 1, w zeta(alpha) for alpha > 1."""
    from scipy.special import zeta
    r = [pump.build_pump(n, 1.0, 0.5).lam_max / n ** 0.5 for n in (400, 1600)]
    assert abs(r[1] / r[0] - 1.0) < 0.1
    r = [pump.build_pump(n, 1.0, 1.0).lam_max / np.log(n) for n in (400, 1600)]
    assert abs(r[1] / r[0] - 1.0) < 0.15
    lm = pump.build_pump(1600, 1.0, 3.0).lam_max
    # an infinite chain's symbol max is 2 zeta(alpha) - 1; the finite open chain approaches it
    assert 1.0 < lm <= 2 * zeta(3.0) - 1 + 1e-12 and lm > 0.99 * (2 * zeta(3.0) - 1)


def test_sylvester_factor_derivative():
    n, w, alpha = 24, 1.7, 0.8
    p = pump.build_pump(n, w, alpha)
    dW = pump.dpump_dalpha(n, w, alpha)
    X = pump.dfactor(p, dW)
    assert np.max(np.abs(p.F @ X + X @ p.F - dW)) < 1e-12 * np.max(np.abs(dW)) * n
    h = 1e-5
    fd = (pump.build_pump(n, w, alpha + h).F - pump.build_pump(n, w, alpha - h).F) / (2 * h)
    assert np.allclose(X, fd, atol=1e-8)
    fdw = (pump.build_pump(n, w + h, alpha).F - pump.build_pump(n, w - h, alpha).F) / (2 * h)
    assert np.allclose(p.F / (2 * w), fdw, atol=1e-8)


def test_invalid_inputs():
    for args in [(0, 1.0, 1.0), (4, -1.0, 1.0), (4, 1.0, -0.5), (4, np.nan, 1.0)]:
        with pytest.raises(ValueError):
            pump.build_pump(*args)
