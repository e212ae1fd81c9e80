"""Pins of the oracle's protocol helpers: the paper's step criterion and
preparation times, the normalised pump, and the root finder (against a
library root of an exact closed form)."""
import math

import numpy as np
from scipy.optimize import brentq

from oracle import closed_forms, observables, protocol, pump


def test_step_criterion_and_times():
    N, gamma = 40, 1.0
    for alpha, w in ((0.5, 2.0), (1.5, 3.0), (0.0, 0.7)):
        p = pump.build_pump(N, w, alpha)
        pr = protocol.protocol(N, w, alpha, gamma, cfl=0.04)
        assert abs(pr.dt * max(gamma * N, p.lam_max) - 0.04) < 1e-15
        assert pr.dt * max(gamma * N, p.lam_max) < 0.05
        assert pr.tau_s == (10.0 / gamma if alpha < 1 else 10.0 / p.lam_min)
        assert pr.tau == 5.0
        assert (pr.n_prep - 1) * pr.dt < pr.tau_s <= pr.n_prep * pr.dt + 1e-12
        assert (pr.n_window - 1) * pr.dt < pr.tau <= pr.n_window * pr.dt + 1e-12
        assert abs(pr.wt - p.lam_max / (gamma * N)) < 1e-15


def test_finite_size_preparation_time_uses_eta():
    """alpha = 1: eta(1) = ln 2, so tau_s = 10 / (w (2 ln 2 - 1))."""
    pr = protocol.protocol(30, 2.5, 1.0, finite_size=True)
    assert abs(pr.tau_s - 10.0 / (2.5 * (2 * math.log(2) - 1))) < 1e-9


def test_normalised_pump_is_linear_in_w():
    a = protocol.protocol(25, 1.3, 0.8)
    b = protocol.protocol(25, 2.6, 0.8)
    assert abs(b.wt - 2 * a.wt) < 1e-13


def test_bisection_root_of_exact_alpha0_law():
    """alpha = 0: <S+S->/N of the exact stationary law crosses 1 at one w;
    bisection agrees with SciPy's Brent root of the same closed form."""
    n, gamma = 10, 1.0

    def f(w):
        return observables.derived(closed_forms.stationary_alpha0(n, gamma, w))[1] / n

    r1 = protocol.bisect(f, 0.05, 0.99, 1.0, tol=1e-12)
    r2 = brentq(lambda w: f(w) - 1.0, 0.05, 0.99, xtol=1e-14)
    assert abs(r1 - r2) < 1e-10
    assert abs(f(r1) - 1.0) < 1e-8
