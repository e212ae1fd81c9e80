"""Brute-force Lindblad master equation of Eq. (1) for tiny N (test only).

L rho = Gamma/2 (2 S- rho S+ - {S+ S-, rho})
        + sum_ij w_ij/2 (2 sigma+_j rho sigma-_i - {sigma-_i sigma+_j, rho})

with sigma^pm = (sigma^x +- i sigma^y)/2 and S^mu = sum_i sigma^mu_i (Model
section).  Basis per site: index 0 = excited (sigma^z = +1), 1 = ground.
Used to pin the oracle's equations of motion at t = 0 and, for N <= 6, to
compare steady states within the TWA error band.
"""
from __future__ import annotations

import numpy as np


def _site_op(op, i, n):
    out = np.array([[1.0 + 0j]])
    for k in range(n):
        out = np.kron(out, op if k == i else np.eye(2))
    return out


def operators(n):
    sp = np.array([[0, 1], [0, 0]], dtype=np.complex128)   # |e><g|
    sz = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    sig_p = [_site_op(sp, i, n) for i in range(n)]
    sig_m = [s.conj().T for s in sig_p]
    sig_z = [_site_op(sz, i, n) for i in range(n)]
    return sig_p, sig_m, sig_z


def lindblad_rhs(rho, W, gamma, ops, decay=None):
    """Right-hand side of Eq. (1).  With ``decay`` (an N x N matrix G) the
    collective term is replaced by correlated decay,
    sum_ab G_ab/2 (2 sigma-_b rho sigma+_a - {sigma+_a sigma-_b, rho})
    (G = Gamma * ones gives the collective term back)."""
    sig_p, sig_m, _ = ops
    n = len(sig_p)
    if decay is None:
        Sp = sum(sig_p)
        Sm = sum(sig_m)
        out = 0.5 * gamma * (2 * Sm @ rho @ Sp - Sp @ Sm @ rho - rho @ Sp @ Sm)
    else:
        out = np.zeros_like(rho)
        for a in range(n):
            for b in range(n):
                if decay[a, b] == 0:
                    continue
                A = sig_p[a] @ sig_m[b]
                out += 0.5 * decay[a, b] * (2 * sig_m[b] @ rho @ sig_p[a] - A @ rho - rho @ A)
    for i in range(n):
        for j in range(n):
            if W[i, j] == 0:
                continue
            A = sig_m[i] @ sig_p[j]
            out += 0.5 * W[i, j] * (2 * sig_p[j] @ rho @ sig_m[i] - A @ rho - rho @ A)
    return out


def liouvillian(W, gamma, n):
    """Superoperator acting on row-major vec(rho)."""
    ops = operators(n)
    d = 2 ** n
    Lm = np.zeros((d * d, d * d), dtype=np.complex128)
    for c in range(d * d):
        e = np.zeros(d * d, dtype=np.complex128)
        e[c] = 1.0
        Lm[:, c] = lindblad_rhs(e.reshape(d, d), W, gamma, ops).reshape(-1)
    return Lm


def product_state(n, up: bool):
    d = 2 ** n
    rho = np.zeros((d, d), dtype=np.complex128)
    idx = 0 if up else d - 1
    rho[idx, idx] = 1.0
    return rho


def expect(rho, op):
    return complex(np.trace(rho @ op))


def steady_state(W, gamma, n, rho0):
    """Long-time state reached from rho0 (propagated to t = 8192 / Gamma)."""
    import scipy.linalg as sla
    Lm = liouvillian(W, gamma, n)
    # propagator over one time unit, squared 13 times: t = 8192 / Gamma
    P = sla.expm(Lm * 1.0)
    for _ in range(13):
        P = P @ P
    v = P @ rho0.reshape(-1)
    d = 2 ** n
    return v.reshape(d, d)
