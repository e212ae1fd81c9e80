"""Pins of the oracle's Toeplitz fast path (circulant embedding of Eq. (2))."""
import itertools

import numpy as np
import pytest
from scipy.linalg import circulant

from oracle import lindblad, pump, toeplitz, twa
from tests.inputs import random_spins


@pytest.mark.parametrize("N", [1, 2, 7, 129, 130, 1000])
@pytest.mark.parametrize("alpha", [0.0, 0.1, 0.5, 1.0, 2.0, 3.0])
def test_embedding_block_spectrum_and_drift(N, alpha):
    """The leading N x N block of the circulant is Eq. (2); its spectrum is
    nonnegative (convex decreasing first column, Dietrich-Newsam); the FFT
    product equals the dense product."""
    w = 1.7
    tp = toeplitz.ToeplitzPump(N, w, alpha)
    W = pump.pump_matrix(N, w, alpha)
    assert tp.M >= 2 * N - 2 and tp.M >= 256 and tp.M & (tp.M - 1) == 0
    if tp.M <= 4096:
        C = circulant(tp.c)
        assert np.array_equal(C[:N, :N], W)
        assert np.allclose(np.sort(np.linalg.eigvalsh(C)), np.sort(tp.lam), atol=1e-10 * tp.lam.max())
    assert tp.lam.min() > -1e-10 * tp.lam.max()
    v = random_spins(3, 4, N)[0]
    ref = v @ W.T
    assert np.max(np.abs(tp.apply(v) - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    vc = random_spins(4, 4, N)
    zc = vc[0] + 1j * vc[1]
    refc = zc @ W.T
    assert np.max(np.abs(tp.apply(zc) - refc)) < 1e-12 * max(1.0, np.max(np.abs(refc)))


def test_zero_padding_would_not_be_psd():
    """Why the law is extended instead of zero padded: a zero-padded embedding
    of Eq. (2) has negative eigenvalues (so the extension is what the pin
    above checks)."""
    N, M = 200, 1024
    c = np.zeros(M)
    c[:N] = pump.pump_matrix(N, 1.0, 0.1)[0]
    c[M - N + 1:] = c[1:N][::-1]
    assert np.fft.fft(c).real.min() < -1e-3


def test_noise_covariance_is_the_pump():
    """Re eta and Im eta of the circulant noise are independent N(0, W)
    (sample covariance over 40000 trajectories within 6 standard errors)."""
    N, B = 6, 40000
    tp = toeplitz.ToeplitzPump(N, 0.9, 1.2)
    W = pump.pump_matrix(N, 0.9, 1.2)
    ex, ey = tp.noise(tp.normals(seed=3, step=5, n_traj=B))
    se = np.sqrt((np.outer(np.diag(W), np.diag(W)) + W ** 2) / B)
    for e in (ex, ey):
        assert np.max(np.abs(e.T @ e / B - W) / se) < 6.0
    assert np.max(np.abs(ex.T @ ey / B) / np.sqrt(np.outer(np.diag(W), np.diag(W)) / B)) < 6.0


def test_normals_slot_layout():
    """eps_k and eps_{k + M/2} come from one Philox call (words (x, y), (z, w))."""
    tp = toeplitz.ToeplitzPump(10, 1.0, 1.0)
    eps = tp.normals(seed=7, step=2, n_traj=3)
    from oracle import philox
    k0, k1 = philox.seed_key(7)
    x = philox.philox4x32_10(5, 1, 2, toeplitz.TAG_CIRCULANT, k0, k1)
    a, b = philox.box_muller(x[0], x[1])
    c, d = philox.box_muller(x[2], x[3])
    assert eps[1, 5] == a + 1j * b and eps[1, 5 + tp.M // 2] == c + 1j * d
    assert abs(np.mean(np.abs(eps) ** 2) - 2.0) < 0.1


def test_noiseless_run_equals_dense_path():
    n, B = 37, 5
    s0 = tuple(random_spins(8, B, n))
    base = dict(n_spin=n, w=2.2, alpha=0.8, n_traj=B, dt=1e-3, n_steps=150, noise=False, init_state=s0, burnin=50)
    a = twa.run(twa.RunConfig(**base))
    b = twa.run(twa.RunConfig(toeplitz=True, **base))
    for u, v in zip(a.final_state, b.final_state):
        assert np.max(np.abs(u - v)) < 1e-12


def _bits_states(n, s0z):
    for bits in itertools.product((-1.0, 1.0), repeat=2 * n):
        yield np.array(bits[:n]), np.array(bits[n:]), np.full(n, s0z)


@pytest.mark.parametrize("up", [True, False])
def test_sz_rate_at_t0_matches_lindblad(up):
    """d<S^z>/dt at t = 0 with the circulant noise equals the exact Lindblad
    rate of Eq. (1) (enumeration of the initial law, exact degree-3 cubature
    over the 2M normals of eps)."""
    n, gamma, w, alpha = 2, 0.8, 1.3, 0.6
    tp = toeplitz.ToeplitzPump(n, w, alpha)
    W = pump.pump_matrix(n, w, alpha)
    ops = lindblad.operators(n)
    rate_q = lindblad.expect(lindblad.lindblad_rhs(lindblad.product_state(n, up), W, gamma, ops), sum(ops[2])).real
    dt, M = 1e-7, tp.M
    d = 2 + 2 * M
    tot, cnt = 0.0, 0
    for x, y, z in _bits_states(n, 1.0 if up else -1.0):
        st = (x[None, :], y[None, :], z[None, :])
        pts = []
        for k in range(d):
            for sg in (1.0, -1.0):
                v = np.zeros(d)
                v[k] = sg * np.sqrt(d)
                pts.append(v)
        P = np.array(pts)
        eps = P[:, 2:2 + M] + 1j * P[:, 2 + M:]
        ex, ey = tp.noise(eps)
        S = tuple(np.repeat(a, len(P), axis=0) for a in st)
        dxi = (np.sqrt(gamma * dt) * P[:, 0], np.sqrt(gamma * dt) * P[:, 1])
        new, _ = twa.heun_step(S, tp, gamma, dt, dxi, (np.sqrt(dt) * ex, np.sqrt(dt) * ey))
        tot += (new[2] - S[2]).sum()
        cnt += len(P)
    assert abs(tot / cnt / dt - rate_q) < 1e-4 * abs(rate_q)


def test_determinism_and_subsets():
    cfg = dict(n_spin=9, w=1.5, alpha=1.1, dt=2e-3, n_steps=30, seed=4, toeplitz=True)
    full = twa.run(twa.RunConfig(n_traj=6, **cfg))
    again = twa.run(twa.RunConfig(n_traj=6, **cfg))
    assert np.array_equal(full.traj_moments, again.traj_moments)
    idx = np.array([5, 1])
    sub = twa.run(twa.RunConfig(n_traj=2, traj=idx, **cfg))
    for c in range(3):
        assert np.array_equal(sub.final_state[c], full.final_state[c][idx])
