"""Correlated decay (oracle, FP64; test infrastructure only).

The paper's model has collective decay Gamma (rank one, all pairs); its
Perspectives note that the TWA evolves an arbitrary correlated-decay matrix of
a Lindbladian at unchanged cost, and SM Sec. S1 step 6 prints the four-point
function needed for correlated emission.  Here, with a symmetric PSD decay
matrix G_ab (Gamma_ab of the SM):

* Eq. (S1) with the collective terms generalised: the deterministic field
  (1/2) Gamma S^a becomes (1/2) (G s^a)_i and the collective noise xi^a becomes
  a correlated noise with <xi_i xi_j> = G_ij, drawn as sqrt(dt) (R zeta') with
  R the PSD square root of G and zeta' standard normals (Philox tag 3, same
  slot layout as the pump noise);
* intensity <sum_ab G_ab s+_a s-_b> = <E2>_TWA + (1/2) sum_a G_aa <s^z_a>_TWA
  with E2 = sum_ab G_ab s+_a s-_b (the single-site correction of step 6: only
  a = b fails to commute; at G_ab = Gamma it is step 6's <S+S-> formula);
* four-point function exactly as printed in SM Sec. S1 step 6; g2 = four-point
  / intensity^2.

Reading (equal in law, not pathwise): the correlated decay noise and the pump
noise are independent Gaussians entering h as xi - chi, so their sum is one
Gaussian of covariance (G + W) dt; it is drawn as -sqrt(dt) C zeta with C the
PSD square root of W + G and zeta the pump's standard normals.  The step is
then Eq. (S1) with the drift matrix W - G, the noise factor C and no
collective term -- the same two contractions per stage as the collective
model, at unchanged cost.  For G = Gamma * ones the drift is identical to the
collective model's and the noise has the same law.

Per trajectory and observed step the estimator needs the nine quantities
  E2, E2^2, E2 D, Q3, R, D^2, U, V, D
with D = sum_a G_aa z_a, Q3 = sum_abc G_ab G_bc s+_a s-_c z_b,
R = sum_a G_aa^2 z_a, U = sum_ab G_ab G_ba z_a z_b, V = sum_ab G_aa G_ab s+_a s-_b
(s+- = (s^x +- i s^y)/2; all real for symmetric G).
"""
from __future__ import annotations

import numpy as np

from .pump import Pump

GEN_NAMES = ("E2", "E2E2", "E2D", "Q3", "R", "DD", "U", "V", "D")


def factor(M: np.ndarray) -> np.ndarray:
    """Symmetric PSD square root of a symmetric PSD matrix (eigenvalues within
    round-off of zero clamped to zero, as for the pump)."""
    lam, V = np.linalg.eigh(M)
    tol = 8.0 * M.shape[0] * np.finfo(np.float64).eps * max(float(lam[-1]), 0.0)
    lam = np.where(lam > tol, lam, 0.0)
    R = (V * np.sqrt(lam)) @ V.T
    return 0.5 * (R + R.T)


class Exchange:
    """Drift matrix with coherent exchange H = sum_{i != j} Omega_ij s+_i s-_j
    (Omega real symmetric, zero diagonal; the coherent dipole-dipole part of
    the Green-tensor kernels named in the Perspectives, which prints no
    equations for it).  Heisenberg's equation for Pauli spins gives
    d s^x_i = s^z_i (Omega s^y)_i dt, d s^y_i = -s^z_i (Omega s^x)_i dt,
    d s^z_i = (s^y_i (Omega s^x)_i - s^x_i (Omega s^y)_i) dt, i.e. s_i x b_i
    with b_i = -(Omega s^x, Omega s^y, 0)_i: in the field of Eq. (S1) it adds
    +dt (Omega s^y)_i to h^x_i and -dt (Omega s^x)_i to h^y_i."""

    def __init__(self, W: np.ndarray, omega: np.ndarray):
        self.W = np.asarray(W, dtype=np.float64)
        self.omega = np.asarray(omega, dtype=np.float64)
        if self.omega.shape != self.W.shape or np.any(np.diag(self.omega) != 0) or \
                not np.array_equal(self.omega, self.omega.T):
            raise ValueError("Omega must be symmetric with a zero diagonal, of the size of W")

    def apply(self, v):
        return v @ self.W.T


def model_pump(W: np.ndarray, G: np.ndarray) -> Pump:
    """Matrices of the correlated-decay step: drift W - G, noise factor
    sqrt(W + G) (eigen-decomposition of W + G, clamped as for the pump)."""
    W = np.asarray(W, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    if W.shape != G.shape or W.shape[0] != W.shape[1]:
        raise ValueError("W and G must be square matrices of one size")
    M = W + G
    lam, V = np.linalg.eigh(M)
    return Pump(W.shape[0], float("nan"), float("nan"), W - G, factor(M), lam, V, float(lam[0]), float(lam[-1]))


def general_quantities(state, G: np.ndarray) -> np.ndarray:
    """The nine per-trajectory quantities of the correlated-emission estimator,
    (n_traj, 9), from the state (x, y, z) each (n_traj, N).  The index sums
    are grouped into matrix-vector products: (G s-)_a = sum_b G_ab s-_b and
    (G^T s+)_b = sum_a G_ab s+_a."""
    x, y, z = state
    sp = 0.5 * (x + 1j * y)
    sm = 0.5 * (x - 1j * y)
    dg = np.diag(G)
    Gsm = sm @ G.T               # (G s-)_a
    GTsp = sp @ G                # (G^T s+)_b
    E2 = np.sum(sp * Gsm, axis=1).real
    D = z @ dg
    Q3 = np.sum(z * GTsp * Gsm, axis=1).real
    R = z @ (dg * dg)
    U = np.sum(z * (z @ (G * G.T).T), axis=1)
    V = np.sum(dg * sp * Gsm, axis=1).real
    return np.stack([E2, E2 * E2, E2 * D, Q3, R, D * D, U, V, D], axis=1)


def derived(m):
    """(intensity, g2) from the ensemble means of the nine quantities."""
    E2, E2E2, E2D, Q3, R, DD, U, V, D = m
    inten = E2 + 0.5 * D
    num = E2E2 + E2D + Q3 - R / 3.0 + 0.25 * (DD + U) - (4.0 / 3.0) * V
    with np.errstate(divide="ignore", invalid="ignore"):
        return inten, num / (inten * inten)


def finalize(traj_gen: np.ndarray):
    """Intensity and g2 of correlated emission with delete-one-block jackknife
    errors (the blocks of the collective observables)."""
    B = traj_gen.shape[0]
    J = min(32, B)
    blk = (np.arange(B) * J) // B
    bsum = np.zeros((J, 9))
    np.add.at(bsum, blk, traj_gen)
    bcnt = np.bincount(blk, minlength=J).astype(np.float64)
    mean = bsum.sum(0) / B
    inten, g2 = derived(mean)
    out = {"I": float(inten), "g2": float(g2)}
    if J >= 2:
        loo = (bsum.sum(0)[None, :] - bsum) / (B - bcnt)[:, None]
        vals = np.stack(derived(loo.T), axis=1)
        se = np.sqrt((J - 1) / J * ((vals - vals.mean(0)) ** 2).sum(0))
        out["I_se"], out["g2_se"] = float(se[0]), float(se[1])
    else:
        out["I_se"] = out["g2_se"] = float("nan")
    return out
