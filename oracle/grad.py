"""Pathwise (fixed-noise) parameter derivatives in FP64 (oracle; test only).

The paper computes no gradients; this module defines what the adjoint of the
HIP library must reproduce.  With the Philox stream held fixed, every
trajectory is a smooth function of (w, alpha) through the pump matrix of
Eq. (2) and its PSD square root F.  Derivatives are propagated forward
(tangent-linear) alongside the Heun steps of ``oracle.twa``:

* dW/dw = W / w, dW/dalpha = -log(1 + |i-j|) W      (Eq. (2));
* dF/dw = F / (2 w); dF/dalpha solves F X + X F = dW/dalpha (``pump.dfactor``);
* the observables' derivatives follow from the chain rule on the time- and
  ensemble-averaged moments; g2 by the quotient rule on the averages.

``fd_gradients`` gives the central finite differences at identical Philox
streams used to cross-check.  ``heun_step_vjp`` is the transpose of the
tangent-linear Heun step (reverse mode), the operation the library's reverse
sweep applies step by step; the dot-product identity <u, J v> = <J^T u, v>
against ``twa.heun_step_tangent`` pins it.
"""
from __future__ import annotations

import numpy as np

from . import observables, philox
from .pump import build_pump, dfactor, dpump_dalpha
from .twa import RunConfig, initial_state, moments, collective_sums


def _incr(state, W, F, gamma, dt, g, zeta, dW=None, dF=None, tang=None):
    x, y, z = state
    sg, sq = np.sqrt(gamma * dt), np.sqrt(dt)
    Sx = x.sum(1)[:, None]
    Sy = y.sum(1)[:, None]
    hx = (0.5 * gamma * Sx - 0.5 * (x @ W.T)) * dt + sg * g[0][:, None] - sq * (zeta[0] @ F.T)
    hy = (0.5 * gamma * Sy - 0.5 * (y @ W.T)) * dt + sg * g[1][:, None] - sq * (zeta[1] @ F.T)
    d = (z * hx, z * hy, -(x * hx + y * hy))
    if tang is None:
        return d, None
    ax, ay, az = tang
    dhx = (0.5 * gamma * ax.sum(1)[:, None] - 0.5 * (ax @ W.T) - 0.5 * (x @ dW.T)) * dt - sq * (zeta[0] @ dF.T)
    dhy = (0.5 * gamma * ay.sum(1)[:, None] - 0.5 * (ay @ W.T) - 0.5 * (y @ dW.T)) * dt - sq * (zeta[1] @ dF.T)
    dd = (az * hx + z * dhx, az * hy + z * dhy, -(ax * hx + x * dhx + ay * hy + y * dhy))
    return d, dd


def _dmoments(state, tang):
    Sx, Sy, Sz = collective_sums(*state)
    dSx, dSy, dSz = (t.sum(1) for t in tang)
    T2 = 0.25 * (Sx * Sx + Sy * Sy)
    dT2 = 0.5 * (Sx * dSx + Sy * dSy)
    return np.stack([dT2, dT2 * Sz + T2 * dSz, 2 * T2 * dT2, dSz, 2 * Sz * dSz], axis=1)


def _dderived(m, dm):
    T2, T3, T4, Z, ZZ = m
    dT2, dT3, dT4, dZ, dZZ = dm
    den = T2 + 0.5 * Z
    num = T4 + 2 * T3 - Z / 3 + 0.5 * ZZ - 4.0 / 3.0 * T2
    dden = dT2 + 0.5 * dZ
    dnum = dT4 + 2 * dT3 - dZ / 3 + 0.5 * dZZ - 4.0 / 3.0 * dT2
    g2 = num / den ** 2
    return dZ, dden, dnum / den ** 2 - 2.0 * g2 * dden / den


def pathwise_gradients(cfg: RunConfig):
    """Returns dict with the observables and d/dw, d/dalpha of (Sz, SpSm, g2)."""
    p = build_pump(cfg.n_spin, cfg.w, cfg.alpha)
    dW = {"w": p.W / cfg.w, "alpha": dpump_dalpha(cfg.n_spin, cfg.w, cfg.alpha)}
    dF = {"w": p.F / (2.0 * cfg.w), "alpha": dfactor(p, dW["alpha"])}
    B, n = cfg.n_traj, cfg.n_spin
    burn = cfg.resolved_burnin()
    state = initial_state(cfg.seed, B, n, cfg.s0z, cfg.point, cfg.traj)
    tang = {k: tuple(np.zeros((B, n)) for _ in range(3)) for k in dW}
    acc = np.zeros((B, 5))
    dacc = {k: np.zeros((B, 5)) for k in dW}
    ns = 0
    for step in range(cfg.n_steps):
        g = philox.collective_noise(cfg.seed, step, B, cfg.point, cfg.traj)
        zeta = philox.pump_noise(cfg.seed, step, B, n, cfg.point, cfg.traj)
        d1, _ = _incr(state, p.W, p.F, cfg.gamma, cfg.dt, g, zeta)
        pred = tuple(s + d for s, d in zip(state, d1))
        d2, _ = _incr(pred, p.W, p.F, cfg.gamma, cfg.dt, g, zeta)
        new_tang = {}
        for k in dW:
            _, t1 = _incr(state, p.W, p.F, cfg.gamma, cfg.dt, g, zeta, dW[k], dF[k], tang[k])
            tp = tuple(a + b for a, b in zip(tang[k], t1))
            _, t2 = _incr(pred, p.W, p.F, cfg.gamma, cfg.dt, g, zeta, dW[k], dF[k], tp)
            new_tang[k] = tuple(a + 0.5 * (b + c) for a, b, c in zip(tang[k], t1, t2))
        state = tuple(s + 0.5 * (a + b) for s, a, b in zip(state, d1, d2))
        tang = new_tang
        if step + 1 > burn:
            acc += moments(state)
            for k in dW:
                dacc[k] += _dmoments(state, tang[k])
            ns += 1
    m = (acc / ns).mean(0)
    out = observables.finalize(acc / ns)
    for k in dW:
        dm = (dacc[k] / ns).mean(0)
        dSz, dSpSm, dg2 = _dderived(m, dm)
        out["d_Sz_d" + k] = float(dSz)
        out["d_SpSm_d" + k] = float(dSpSm)
        out["d_g2_d" + k] = float(dg2)
    return out


def fd_gradients(cfg: RunConfig, h: float = 1e-4, params=("w", "alpha")):
    """Central differences of (Sz, SpSm, g2) in w and alpha at fixed noise."""
    from dataclasses import replace
    from .twa import run
    out = {}
    for k in params:
        vals = []
        for sgn in (+1, -1):
            c = replace(cfg, **{k: getattr(cfg, k) + sgn * h})
            vals.append(observables.finalize(run(c).traj_moments))
        for name in ("Sz", "SpSm", "g2"):
            out["d_%s_d%s" % (name, k)] = (vals[0][name] - vals[1][name]) / (2 * h)
    return out


def _incr_vjp(state, mu, fields_dt, W, gamma, dt):
    """Transpose of the linearisation of one increment of Eq. (S1) at ``state``
    with fixed noise: cotangent ``mu`` = (mu^x, mu^y, mu^z) of the increment
    f = (s^z H^x, s^z H^y, -(s^x H^x + s^y H^y)), H^a the dt-scaled fields
    ``fields_dt``, returns the cotangent of the state.  The fields depend on
    the state through H^a_i = (Gamma/2 sum_j s^a_j - 1/2 sum_j w_ij s^a_j) dt + noise."""
    x, y, z = state
    hx, hy = fields_dt
    ux, uy, uz = mu
    # direct dependence of f on s at fixed H
    cx = -uz * hx
    cy = -uz * hy
    cz = ux * hx + uy * hy
    # dependence through H: nu^a = (df/dH^a)^T mu
    nx = ux * z - uz * x
    ny = uy * z - uz * y
    cx = cx + (0.5 * gamma * nx.sum(axis=1)[:, None] - 0.5 * (nx @ W)) * dt
    cy = cy + (0.5 * gamma * ny.sum(axis=1)[:, None] - 0.5 * (ny @ W)) * dt
    return cx, cy, cz


def heun_step_vjp(state, cot, W, gamma, dt, dxi, dchi):
    """Reverse mode of one stochastic Heun step s' = s + (f(s) + f(s + f(s)))/2
    at fixed noise: the cotangent of s' -> the cotangent of s."""
    from .twa import heun_step
    _, (d1, pred, d2) = heun_step(state, W, gamma, dt, dxi, dchi)
    mu2 = tuple(0.5 * c for c in cot)
    lam_pred = _incr_vjp(pred, mu2, d2[3], W, gamma, dt)
    mu1 = tuple(0.5 * c + lp for c, lp in zip(cot, lam_pred))
    lam_s = _incr_vjp(state, mu1, d1[3], W, gamma, dt)
    return tuple(c + lp + ls for c, lp, ls in zip(cot, lam_pred, lam_s))
