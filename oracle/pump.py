"""Pump-rate matrix, channel decomposition and noise factor (oracle, FP64).

Test infrastructure only; see the package docstring.

* Eq. (2): w_ij = w / (|i - j| + 1)^alpha on an open chain (indices 0..N-1).
* Main text after Eq. (2): the pump splits into N channels whose rates are the
  eigenvalues of w_ij; the normalised pump is w~ = w_max / (Gamma N), with
  w_max from numerical diagonalisation.
* Main text after Eq. (3): the smallest channel rate is approximately
  w (2 eta(alpha) - 1), eta the Dirichlet eta function.
* Eq. (S1) noise: <chi_i chi_j> = w_ij.  Any F with F F^T = W has that law; the
  reading used on both sides is the unique symmetric positive-semidefinite
  square root F = V diag(sqrt(lambda+)) V^T, defined also at alpha = 0 where W
  has rank one; lambda+ is lambda where lambda > 8 N eps lambda_max (eps the
  binary64 unit round-off) and 0 otherwise, so that round-off eigenvalues of
  the rank-one case do not leak sqrt(eps)-sized noise into F.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def pump_matrix(n_spin: int, w: float, alpha: float) -> np.ndarray:
    """Eq. (2) on an open chain."""
    i = np.arange(n_spin)
    d = np.abs(i[:, None] - i[None, :]).astype(np.float64)
    return w / (d + 1.0) ** alpha


def dpump_dalpha(n_spin: int, w: float, alpha: float) -> np.ndarray:
    """d w_ij / d alpha = -log(1 + |i-j|) w_ij (derivative of Eq. (2))."""
    i = np.arange(n_spin)
    d = np.abs(i[:, None] - i[None, :]).astype(np.float64)
    return -np.log1p(d) * w / (d + 1.0) ** alpha


@dataclass
class Pump:
    n_spin: int
    w: float
    alpha: float
    W: np.ndarray          # (N, N) Eq. (2)
    F: np.ndarray          # (N, N) symmetric PSD square root of W
    lam: np.ndarray        # eigenvalues of W, ascending
    V: np.ndarray          # eigenvectors (columns)
    lam_min: float
    lam_max: float


def build_pump(n_spin: int, w: float, alpha: float) -> Pump:
    """Channel decomposition of Eq. (2) and the PSD noise factor."""
    if n_spin < 1 or not np.isfinite(w) or not np.isfinite(alpha) or w < 0 or alpha < 0:
        raise ValueError("need N >= 1, finite w >= 0, finite alpha >= 0")
    W = pump_matrix(n_spin, w, alpha)
    lam, V = np.linalg.eigh(W)
    # eigenvalues within round-off of zero (the rank-one alpha = 0 case) are zero
    tol = 8.0 * n_spin * np.finfo(np.float64).eps * max(float(lam[-1]), 0.0)
    lam_c = np.where(lam > tol, lam, 0.0)
    F = (V * np.sqrt(lam_c)) @ V.T
    F = 0.5 * (F + F.T)
    return Pump(n_spin, float(w), float(alpha), W, F, lam, V, float(lam[0]), float(lam[-1]))


def build_pump_dense(W: np.ndarray) -> Pump:
    """Channel decomposition and PSD noise factor of an arbitrary symmetric PSD
    pump matrix (the general pump of the Perspectives), with the same square
    root as ``build_pump``; w and alpha are recorded as NaN."""
    W = np.array(W, dtype=np.float64)
    n = W.shape[0]
    if W.shape != (n, n) or not np.all(np.isfinite(W)) or np.max(np.abs(W - W.T)) > 0:
        raise ValueError("need a finite symmetric square matrix")
    lam, V = np.linalg.eigh(W)
    if lam[0] < -1e-10 * max(float(lam[-1]), 0.0):
        raise ValueError("pump matrix is not positive semidefinite")
    tol = 8.0 * n * np.finfo(np.float64).eps * max(float(lam[-1]), 0.0)
    lam_c = np.where(lam > tol, lam, 0.0)
    F = (V * np.sqrt(lam_c)) @ V.T
    F = 0.5 * (F + F.T)
    return Pump(n, float("nan"), float("nan"), W, F, lam, V, float(lam[0]), float(lam[-1]))


def normalised_pump(p: Pump, gamma: float = 1.0) -> float:
    """w~ = w_max / (Gamma N) (main text, after Eq. (3))."""
    return p.lam_max / (gamma * p.n_spin)


def dirichlet_eta(alpha: float, terms: int = 200000) -> float:
    """eta(alpha) = sum_{m>=1} (-1)^(m-1) / m^alpha, summed in pairs with an
    Euler-type tail average so that it converges for all alpha > 0."""
    m = np.arange(1, terms + 1, dtype=np.float64)
    a = (-1.0) ** (m - 1) / m ** alpha
    s = np.cumsum(a)
    return float(0.5 * (s[-1] + s[-2]))


def lam_min_estimate(w: float, alpha: float) -> float:
    """w (2 eta(alpha) - 1): Toeplitz estimate of the smallest channel rate."""
    return w * (2.0 * dirichlet_eta(alpha) - 1.0)


def dfactor(p: Pump, dW: np.ndarray) -> np.ndarray:
    """Derivative of the PSD square root along dW: solves F X + X F = dW.

    In the eigenbasis of W (F = V diag(r) V^T with r = sqrt(lambda)) the
    Sylvester equation is diagonal: X'_ij = (V^T dW V)_ij / (r_i + r_j),
    set to zero where r_i + r_j = 0.
    """
    tol = 8.0 * p.n_spin * np.finfo(np.float64).eps * max(p.lam_max, 0.0)
    r = np.sqrt(np.where(p.lam > tol, p.lam, 0.0))
    B = p.V.T @ dW @ p.V
    den = r[:, None] + r[None, :]
    Xp = np.where(den > 0, B / np.where(den > 0, den, 1.0), 0.0)
    X = p.V @ Xp @ p.V.T
    return 0.5 * (X + X.T)
