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
