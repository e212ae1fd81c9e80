"""Counter-based noise for the oracle (test infrastructure only).

The paper does not name a random-number generator (SM Sec. S1 only states the
noise covariances of Eq. (S1)).  Reading adopted on both sides of the parity
check: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written here from that paper's definition, then the
Box-Muller transform (Box & Muller 1958).

Counter layout (a reading, identical on the HIP side, implemented there
independently):

* key   = (seed & 0xffffffff, seed >> 32)
* ctr   = (slot, trajectory k, step n, tag | point << 8)
* tag 0 = pump noise of step n: slot m yields 4 words -> two Box-Muller pairs
          (zeta^x_{2m}, zeta^y_{2m}) and (zeta^x_{2m+1}, zeta^y_{2m+1}).
* tag 1 = collective noise of step n: slot 0, first pair -> (g^x, g^y).
* tag 2 = initial signs (step field 0): slot m gives 128 bits covering spins
          64m .. 64m+63; bit 2j of the 128-bit word is the sign of s^x of spin
          64m+j, bit 2j+1 the sign of s^y; a set bit means +1.

Uniforms: u1 = ((x >> 8) + 1) * 2^-24 in (0, 1], u2 = (x >> 8) * 2^-24 in
[0, 1); both are exact in binary32 and binary64.
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
# Multipliers and Weyl key increments of Philox4x32 (Salmon et al. 2011).
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)

TAG_PUMP = 0
TAG_COLLECTIVE = 1
TAG_INIT = 2


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on broadcastable uint32 counter words.

    Each round multiplies words 0 and 2 by the two constants, keeps the 64-bit
    products as (hi, lo), and forms (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key
    is advanced by the Weyl increments between rounds.
    """
    c = [np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & _MASK
            k1 = (k1 + PHILOX_W1) & _MASK
        p0 = PHILOX_M0 * c[0]
        p1 = PHILOX_M1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & _MASK,
             (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & _MASK]
    return [x.astype(np.uint32) for x in c]


def seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def box_muller(a, b):
    """Two standard normals from two uint32 words (Box & Muller 1958)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    u1 = ((a >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24
    u2 = (b >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def _tagword(tag: int, point: int):
    return np.uint64((tag | (int(point) << 8)) & 0xFFFFFFFF)


def _traj_index(n_traj: int, traj):
    """Trajectory counters: 0 .. n_traj-1, or the given trajectory indices."""
    if traj is None:
        return np.arange(n_traj, dtype=np.uint64)
    t = np.asarray(traj, dtype=np.uint64).reshape(-1)
    if t.shape[0] != n_traj:
        raise ValueError("traj must list n_traj trajectory indices")
    return t


def pump_noise(seed: int, step: int, n_traj: int, n_spin: int, point: int = 0, traj=None):
    """Standard normals zeta^x, zeta^y of shape (n_traj, n_spin) for one step
    (of trajectories 0 .. n_traj-1, or of the trajectory indices ``traj``)."""
    k0, k1 = seed_key(seed)
    n_slot = (n_spin + 1) // 2
    m = np.arange(n_slot, dtype=np.uint64)[None, :]
    k = _traj_index(n_traj, traj)[:, None]
    x0, x1, x2, x3 = philox4x32_10(m, k, np.uint64(step), _tagword(TAG_PUMP, point), k0, k1)
    za, zb = box_muller(x0, x1)   # spin 2m: (x, y)
    zc, zd = box_muller(x2, x3)   # spin 2m+1: (x, y)
    zx = np.empty((n_traj, 2 * n_slot))
    zy = np.empty((n_traj, 2 * n_slot))
    zx[:, 0::2], zy[:, 0::2] = za, zb
    zx[:, 1::2], zy[:, 1::2] = zc, zd
    return zx[:, :n_spin], zy[:, :n_spin]


def collective_noise(seed: int, step: int, n_traj: int, point: int = 0, traj=None):
    """Standard normals g^x, g^y of shape (n_traj,) for one step."""
    k0, k1 = seed_key(seed)
    k = _traj_index(n_traj, traj)
    x0, x1, _, _ = philox4x32_10(np.uint64(0), k, np.uint64(step), _tagword(TAG_COLLECTIVE, point), k0, k1)
    return box_muller(x0, x1)


def initial_signs(seed: int, n_traj: int, n_spin: int, point: int = 0, traj=None):
    """+-1 signs (sx, sy), each (n_traj, n_spin), for the discrete initial sampling."""
    k0, k1 = seed_key(seed)
    n_slot = (n_spin + 63) // 64
    m = np.arange(n_slot, dtype=np.uint64)[None, :]
    k = _traj_index(n_traj, traj)[:, None]
    words = philox4x32_10(m, k, np.uint64(0), _tagword(TAG_INIT, point), k0, k1)
    bits = np.zeros((n_traj, n_slot, 128), dtype=np.int8)
    for w in range(4):
        wv = words[w].astype(np.uint64)
        for b in range(32):
            bits[:, :, 32 * w + b] = ((wv >> np.uint64(b)) & np.uint64(1)).astype(np.int8)
    sx = bits[:, :, 0::2].reshape(n_traj, 64 * n_slot)[:, :n_spin]
    sy = bits[:, :, 1::2].reshape(n_traj, 64 * n_slot)[:, :n_spin]
    return 2.0 * sx - 1.0, 2.0 * sy - 1.0
