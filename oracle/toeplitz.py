"""Toeplitz fast path of the Eq. (2) pump (oracle, FP64; test infrastructure only).

Not in the paper: a second way to apply the pump of Eq. (2) that uses its
Toeplitz structure.  On an open chain w_ij = c(|i - j|) with c(d) =
w / (1 + d)^alpha, a convex decreasing sequence.  Extend the same law to
d <= M/2 and wrap it into a circulant C of size M >= 2N - 2 with first column
c~_j = c(min(j, M - j)); the leading N x N block of C is W.  A positive,
convex, decreasing first column makes the minimal circulant embedding
positive semidefinite (Dietrich and Newsam, SIAM J. Sci. Comput. 18 (1997);
the eigenvalues are lam = DFT(c~), all real), so

* drift: W v = (C [v; 0])[:N] = IDFT(lam * DFT([v; 0]))[:N], with the two
  components packed as v = s^x + i s^y (C is real);
* noise: eta = IDFT(sqrt(lam M) * eps)[:N] with eps_k = a_k + i b_k, a, b
  independent standard normals: Re eta and Im eta are independent N(0, W)
  vectors (the pump noise of s^x and s^y), since
  Cov(Re eta_j, Re eta_l) = Re (1/M) sum_k lam_k e^{2 pi i (j-l) k / M} = c~_{j-l}.

DFT(x)_k = sum_j x_j e^{-2 pi i j k / M}, IDFT its inverse (1/M included).
The noise is equal in law to the dense path's sqrt(dt) F zeta, not pathwise.
Embedding size M = max(256, the smallest power of two >= 2N - 2).
Normals: Philox counter (slot k, trajectory, step, tag 3 | point << 8) for
k < M/2; words (x, y) give eps_k and words (z, w) give eps_{k + M/2}, each by
Box-Muller.
"""
from __future__ import annotations

import numpy as np

from . import philox

TAG_CIRCULANT = 3


def embedding_size(n_spin: int) -> int:
    m = 256
    while m < 2 * n_spin - 2:
        m *= 2
    return m


def first_column(n_spin: int, w: float, alpha: float, M: int = None) -> np.ndarray:
    """c~_j = w / (1 + min(j, M - j))^alpha, j = 0 .. M-1."""
    M = embedding_size(n_spin) if M is None else M
    j = np.arange(M)
    d = np.minimum(j, M - j).astype(np.float64)
    return w / (1.0 + d) ** alpha


def spectrum(c: np.ndarray) -> np.ndarray:
    """Eigenvalues of the circulant with first column c (real: c is symmetric)."""
    return np.fft.fft(c).real


class ToeplitzPump:
    """Eq. (2) applied through the circulant embedding."""

    def __init__(self, n_spin: int, w: float, alpha: float):
        self.n_spin = n_spin
        self.w = float(w)
        self.alpha = float(alpha)
        self.M = embedding_size(n_spin)
        self.c = first_column(n_spin, w, alpha, self.M)
        self.lam = spectrum(self.c)
        # eigenvalues within round-off of zero count as zero (as for the dense factor)
        tol = 8.0 * self.M * np.finfo(np.float64).eps * max(float(self.lam.max()), 0.0)
        self.lam_plus = np.where(self.lam > tol, self.lam, 0.0)

    def apply(self, v: np.ndarray) -> np.ndarray:
        """W v for v of shape (n_traj, N), real or complex."""
        B, n = v.shape
        pad = np.zeros((B, self.M), dtype=np.complex128)
        pad[:, :n] = v
        out = np.fft.ifft(self.lam[None, :] * np.fft.fft(pad, axis=1), axis=1)[:, :n]
        return out.real if np.isrealobj(v) else out

    def normals(self, seed: int, step: int, n_traj: int, point: int = 0, traj=None) -> np.ndarray:
        """eps (n_traj, M) complex standard normals of one step."""
        M = self.M
        k0, k1 = philox.seed_key(seed)
        slot = np.arange(M // 2, dtype=np.uint64)[None, :]
        k = philox._traj_index(n_traj, traj)[:, None]
        tag = np.uint64((TAG_CIRCULANT | (int(point) << 8)) & 0xFFFFFFFF)
        x0, x1, x2, x3 = philox.philox4x32_10(slot, k, np.uint64(step), tag, k0, k1)
        a0, b0 = philox.box_muller(x0, x1)
        a1, b1 = philox.box_muller(x2, x3)
        eps = np.empty((n_traj, M), dtype=np.complex128)
        eps[:, :M // 2] = a0 + 1j * b0
        eps[:, M // 2:] = a1 + 1j * b1
        return eps

    def noise(self, eps: np.ndarray) -> tuple:
        """(Re eta, Im eta)[:, :N] for eps of shape (n_traj, M)."""
        eta = np.fft.ifft(np.sqrt(self.lam_plus * self.M)[None, :] * eps, axis=1)[:, :self.n_spin]
        return eta.real, eta.imag
