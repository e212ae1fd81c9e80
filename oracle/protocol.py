"""The paper's simulation protocol and threshold quantities (oracle; test
infrastructure only).

* Time step: the criterion of the main text's methods paragraph,
  max(Gamma N, lambda_max) dt < 0.05; here dt = cfl / max(Gamma N, lambda_max).
* Preparation time tau_s: 10/Gamma for alpha < 1 and 10/lambda_min for
  alpha >= 1 (main text); with ``finite_size`` the SM's choice
  10 / [w (2 eta(alpha) - 1)] for every alpha (the Toeplitz estimate of the
  slowest pump mode, text after Eq. (3)).
* Window tau = 5/Gamma, over which the observables are also time averaged.
* Normalised pump w~ = lambda_max / (Gamma N) (text after Eq. (2)); lambda_max
  is linear in w at fixed alpha.
* Thresholds (main text, results): g2 <= 1.08 delimits coherent emission,
  <S+S-> > N superradiance; g2_min is the minimum of g2 over equally spaced
  w~ in [1/10, 1].

The root of a fixed-noise objective is found here by plain bisection on the
oracle's own runs, the minimum of g2 by evaluating the scan points.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import observables
from . import pump as opump
from . import twa as otwa


@dataclass
class Protocol:
    dt: float
    tau_s: float
    tau: float
    n_prep: int
    n_window: int
    wt: float
    lam_min: float
    lam_max: float


def protocol(N: int, w: float, alpha: float, gamma: float = 1.0, cfl: float = 0.04, finite_size: bool = False,
             pump=None) -> Protocol:
    p = pump if pump is not None else opump.build_pump(N, w, alpha)
    dt = cfl / max(gamma * N, p.lam_max)
    if finite_size:
        tau_s = 10.0 / (w * (2.0 * opump.dirichlet_eta(alpha) - 1.0))
    elif alpha < 1.0:
        tau_s = 10.0 / gamma
    else:
        tau_s = 10.0 / p.lam_min
    tau = 5.0 / gamma
    return Protocol(dt=dt, tau_s=tau_s, tau=tau, n_prep=int(math.ceil(tau_s / dt - 1e-9)),
                    n_window=int(math.ceil(tau / dt - 1e-9)), wt=p.lam_max / (gamma * N),
                    lam_min=p.lam_min, lam_max=p.lam_max)


def objective(N, w, alpha, n_traj, dt, n_steps, burnin, seed=0, which="g2", gamma=1.0, s0z=1.0):
    """Fixed-noise steady-state objective: g2, or <S+S->/N."""
    cfg = otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=n_traj, dt=dt, n_steps=n_steps, seed=seed,
                         gamma=gamma, s0z=s0z, burnin=burnin)
    m = observables.finalize(otwa.run(cfg).traj_moments)
    return m["g2"] if which == "g2" else m["SpSm"] / N


def bisect(f, lo: float, hi: float, target: float, tol: float = 1e-10, max_iter: int = 200) -> float:
    """Root of f(x) = target in [lo, hi] by bisection (f(lo) - target and
    f(hi) - target of opposite signs)."""
    flo = f(lo) - target
    fhi = f(hi) - target
    if flo * fhi > 0:
        raise ValueError("no sign change on the bracket")
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        fm = f(mid) - target
        if (fm < 0) == (flo < 0):
            lo, flo = mid, fm
        else:
            hi, fhi = mid, fm
        if hi - lo < tol:
            break
    return 0.5 * (lo + hi)


def g2_scan(N, alpha, n_traj, wts, seed=0, gamma=1.0, cfl=0.04, finite_size=False, s0z=1.0):
    """g2 at each normalised pump w~ of ``wts``, each point with its own protocol."""
    lam1 = opump.build_pump(N, 1.0, alpha).lam_max       # lambda_max at w = 1
    out = []
    for wt in wts:
        w = wt * gamma * N / lam1
        pr = protocol(N, w, alpha, gamma, cfl, finite_size)
        T = pr.n_prep + pr.n_window
        out.append(objective(N, w, alpha, n_traj, pr.dt, T, pr.n_prep, seed, "g2", gamma, s0z))
    return np.array(out)
