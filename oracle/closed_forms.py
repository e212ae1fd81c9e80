"""Closed forms at alpha = 0 used to pin the oracle (test infrastructure only).

At alpha = 0, Eq. (2) gives w_ij = w for all i, j, so every spin of a
trajectory sees the same effective field in Eq. (S1) and the collective spin
S = sum_i s_i rotates rigidly: its length R is conserved.

* Noiseless superradiant decay: N identical spins of length r obey
  dz/dt = -kappa (r^2 - z^2) with kappa = (Gamma - w) N / 2, solved by
  z(t) = -r tanh(kappa r (t - t_D)).
* Stationary law with noise: the direction of S diffuses on the sphere of
  radius R with rotational intensity Gamma + w about the x and y axes and
  drifts with angular speed (Gamma - w) R sin(theta) / 2, so u = cos(theta)
  has density proportional to exp(-k u) on [-1, 1], k = (Gamma - w) R / (Gamma + w),
  and uniform azimuth.  R^2 = X^2 + Y^2 + N^2 where X, Y are the sums of the
  initial +-1 transverse components (independent Rademacher sums).  At
  w = Gamma the law is uniform and <S+S-> = (N^2 + 2N)/6, the Dicke value; the
  paper's collective-pump section gives g2 -> 6/5 there as N grows.
* Detailed balance of the exact alpha = 0 steady state in the Dicke manifold
  J = N/2 (SM, collective spin pump): populations p_{m+1} = (w/Gamma) p_m.
"""
from __future__ import annotations

import numpy as np
from math import comb


def noiseless_collective_z(t, n_spin, gamma, w, r, z0):
    kappa = 0.5 * (gamma - w) * n_spin
    tD = np.arctanh(z0 / r) / (kappa * r)
    return -r * np.tanh(kappa * r * (np.asarray(t) - tD))


def _rademacher_sum_law(n):
    vals = np.array([2 * k - n for k in range(n + 1)], dtype=np.float64)
    prob = np.array([comb(n, k) for k in range(n + 1)], dtype=np.float64) / 2.0 ** n
    return vals, prob


def _u_moments(k, nodes, weights):
    """E[u^p] and E[(1-u^2)^q u^p] under density exp(-k u) on [-1,1]."""
    dens = np.exp(-k * nodes - np.max(-k * nodes))
    Z = np.sum(weights * dens)
    E = lambda f: float(np.sum(weights * dens * f) / Z)
    return E


def stationary_alpha0(n_spin: int, gamma: float, w: float):
    """Exact stationary TWA moments (T2, T3, T4, Z, ZZ) at alpha = 0."""
    vals, prob = _rademacher_sum_law(n_spin)
    nodes, weights = np.polynomial.legendre.leggauss(200)
    acc = np.zeros(5)
    for X, pX in zip(vals, prob):
        for Y, pY in zip(vals, prob):
            R = np.sqrt(X * X + Y * Y + n_spin * n_spin)
            k = (gamma - w) * R / (gamma + w)
            E = _u_moments(k, nodes, weights)
            s2 = 1.0 - nodes ** 2
            T2 = R ** 2 * E(s2) / 4.0
            T3 = R ** 3 * E(s2 * nodes) / 4.0
            T4 = R ** 4 * E(s2 ** 2) / 16.0
            Zm = R * E(nodes)
            ZZ = R ** 2 * E(nodes ** 2)
            acc += pX * pY * np.array([T2, T3, T4, Zm, ZZ])
    return acc


def dicke_alpha0(n_spin: int, gamma: float, w: float):
    """Exact quantum steady state at alpha = 0 in the J = N/2 manifold:
    returns (<S^z>, <S+S->, g2) with S^z = 2 J_z and S^+ = J^+."""
    J = 0.5 * n_spin
    m = np.arange(-J, J + 1)
    r = w / gamma
    logp = (m + J) * np.log(r) if r > 0 else np.where(m == -J, 0.0, -np.inf)
    p = np.exp(logp - np.max(logp))
    p /= p.sum()
    jpjm = J * (J + 1) - m * (m - 1)            # <m| J+ J- |m>
    jpjm2 = jpjm * (J * (J + 1) - (m - 1) * (m - 2))
    spsm = float(np.sum(p * jpjm))
    return float(np.sum(p * 2 * m)), spsm, float(np.sum(p * jpjm2)) / spsm ** 2
