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


_ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>
#include <cstdio>
// stdin: records of six uint32 (c0, c1, c2, c3, k0, k1); stdout: the four
// output words of each.  rocRAND's engine keys on the 64-bit seed, puts the
// subsequence in counter words 2..3 and offset / 4 in words 0..1.
int main() {
    uint32_t in[6];
    while (std::fread(in, 4, 6, stdin) == 6) {
        const unsigned long long seed = in[4] | ((unsigned long long)in[5] << 32);
        const unsigned long long sub = in[2] | ((unsigned long long)in[3] << 32);
        const unsigned long long off = 4ull * (in[0] | ((unsigned long long)in[1] << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        const uint4 r = e.next4();
        const uint32_t out[4] = {r.x, r.y, r.z, r.w};
        std::fwrite(out, 4, 4, stdout);
    }
    return 0;
}
"""


def test_philox_matches_rocrand_engine(tmp_path):
    """Cross-implementation check: rocRAND's Philox4x32-10 engine (its
    header, built here for the host and run) gives the oracle's output words
    on random counters and keys and on the carry edges of every word.  Word 1
    stays below 2^30 so that rocRAND's 64-bit number offset (4 per counter)
    does not wrap."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc or the rocRAND headers are not installed")
    src = tmp_path / "philox_rocrand.cpp"
    src.write_text(_ROCRAND_PROBE)
    exe = tmp_path / "philox_rocrand"
    subprocess.run([hipcc, "-O2", "-x", "hip", "--offload-host-only", str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    rng = np.random.default_rng(11)
    n = 1 << 16
    m32 = 0xFFFFFFFF
    edge = np.array([[0, 0, 0, 0], [m32, 0, 0, 0], [m32, 5, m32, m32], [1, 2, 3, 4], [m32, (1 << 30) - 1, m32, m32]],
                    dtype=np.uint64)
    for k0, k1 in [(0, 0), (0xDEADBEEF, 0x12345678), (m32, m32), (7, 0)]:
        c = rng.integers(0, 1 << 32, size=(n, 4), dtype=np.uint64)
        c[:, 1] >>= np.uint64(2)
        c = np.concatenate([edge, c])
        rec = np.empty((c.shape[0], 6), dtype=np.uint32)
        rec[:, :4] = c
        rec[:, 4], rec[:, 5] = k0, k1
        out = subprocess.run([str(exe)], input=rec.tobytes(), check=True, capture_output=True).stdout
        got = np.frombuffer(out, dtype=np.uint32).reshape(-1, 4)
        want = np.stack(philox.philox4x32_10(c[:, 0], c[:, 1], c[:, 2], c[:, 3], k0, k1), axis=1)
        assert np.array_equal(got.astype(np.uint64), want)
