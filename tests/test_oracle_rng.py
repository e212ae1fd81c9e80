"""Pins of the oracle's counter-based noise (Philox4x32-10 + Box-Muller)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(*r[:4], r[4], r[5])
        assert [int(o) for o in out] == r[6:]


def test_philox_vectorised_matches_scalar():
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2 ** 32, size=(4, 64), dtype=np.uint64)
    vec = philox.philox4x32_10(c[0], c[1], c[2], c[3], 0x1234, 0xABCD)
    for j in range(64):
        sc = philox.philox4x32_10(c[0, j], c[1, j], c[2, j], c[3, j], 0x1234, 0xABCD)
        assert [int(v[j]) for v in vec] == [int(s) for s in sc]


def test_box_muller_moments_and_ks():
    k = np.arange(250000, dtype=np.uint64)
    w = philox.philox4x32_10(k, 7, 3, 0, 11, 0)
    z = np.concatenate(philox.box_muller(w[0], w[1]) + philox.box_muller(w[2], w[3]))
    n = z.size
    assert abs(z.mean()) < 4.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * np.sqrt(2.0 / n)
    kurt = np.mean(z ** 4)
    assert abs(kurt - 3.0) < 4.0 * np.sqrt(96.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_uniform_endpoints_exact():
    z0, z1 = philox.box_muller(np.array([0xFFFFFFFF], dtype=np.uint64), np.array([0], dtype=np.uint64))
    # u1 = 1 gives radius 0
    assert z0[0] == 0.0 and z1[0] == 0.0
    z0, _ = philox.box_muller(np.array([0], dtype=np.uint64), np.array([0], dtype=np.uint64))
    assert np.isclose(z0[0], np.sqrt(-2.0 * np.log(2.0 ** -24)))


def test_pump_noise_slot_layout():
    zx, zy = philox.pump_noise(seed=42, step=9, n_traj=3, n_spin=5)
    k0, k1 = philox.seed_key(42)
    for k in range(3):
        for m in range(3):
            w = philox.philox4x32_10(m, k, 9, philox.TAG_PUMP, k0, k1)
            a = philox.box_muller(w[0], w[1])
            b = philox.box_muller(w[2], w[3])
            assert zx[k, 2 * m] == a[0] and zy[k, 2 * m] == a[1]
            if 2 * m + 1 < 5:
                assert zx[k, 2 * m + 1] == b[0] and zy[k, 2 * m + 1] == b[1]


def test_streams_are_distinct_across_tags_points_steps():
    a = philox.pump_noise(1, 0, 4, 8)[0]
    b = philox.pump_noise(1, 1, 4, 8)[0]
    c = philox.pump_noise(1, 0, 4, 8, point=1)[0]
    g = philox.collective_noise(1, 0, 4)[0]
    assert not np.allclose(a, b) and not np.allclose(a, c)
    assert not np.allclose(a[:, 0], g)


def test_initial_signs_balanced_and_bit_layout():
    sx, sy = philox.initial_signs(3, 512, 100)
    assert set(np.unique(sx)) == {-1.0, 1.0}
    n = sx.size
    for arr in (sx, sy):
        assert abs(arr.mean()) < 4.0 / np.sqrt(n)
    assert abs(np.mean(sx * sy)) < 4.0 / np.sqrt(n)
    k0, k1 = philox.seed_key(3)
    w = philox.philox4x32_10(1, 7, 0, philox.TAG_INIT, k0, k1)   # slot 1 covers spins 64..99
    j = 5                                                         # spin 69
    bit_x, bit_y = 2 * j, 2 * j + 1
    assert sx[7, 64 + j] == (1.0 if (int(w[bit_x // 32]) >> (bit_x % 32)) & 1 else -1.0)
    assert sy[7, 64 + j] == (1.0 if (int(w[bit_y // 32]) >> (bit_y % 32)) & 1 else -1.0)
