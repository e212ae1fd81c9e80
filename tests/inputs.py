"""Seeded synthetic inputs shared by the oracle and HIP-path tests.

Holds no arithmetic of the method: only random classical spin states
(directions uniform on the sphere, length sqrt(3) as for the discrete
sampling of SM Sec. S1) for tests that start from non-sampled states.
"""
import numpy as np


def random_spins(seed: int, n_traj: int, n_spin: int) -> np.ndarray:
    """(3, n_traj, n_spin) array of spins of length sqrt(3), uniform directions."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, n_traj, n_spin))
    v *= np.sqrt(3.0) / np.linalg.norm(v, axis=0)
    return v


def free_space_decay(n_spin: int, d_over_lambda: float, gamma0: float = 1.0) -> np.ndarray:
    """Correlated-decay matrix of a chain of emitters with spacing d in free
    space, scalar kernel Gamma_ij = gamma0 sinc(k d |i - j|), k = 2 pi / lambda
    (positive semidefinite for any positions: the Fourier transform of a
    uniform measure on a sphere).  d -> 0 gives collective decay
    gamma0 * ones; d = lambda / 2 gives independent decay gamma0 * identity."""
    i = np.arange(n_spin)
    r = 2.0 * np.pi * d_over_lambda * np.abs(i[:, None] - i[None, :]).astype(np.float64)
    return gamma0 * np.sinc(r / np.pi)


def random_psd(seed: int, n: int, rank: int = None) -> np.ndarray:
    """Random symmetric PSD matrix A A^T / n (rank ``rank``, default full)."""
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n if rank is None else rank))
    return A @ A.T / n
