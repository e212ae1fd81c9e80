"""Parity of the response copies (two-time correlation, Eq. (S3) and the
three-copy response after it) and of the reverse sweep (pathwise gradients)
on the tile configurations the full-size workloads take: 64x64 (tile 1),
128x128 (tiles 2 and 3, the FP64 and N ~ 1000-2000 FP32 path) and 320x256
(tile 7, the FP32 / BF16 path for N >= ~800), at sizes with ragged spin and
trajectory padding, against the FP64 oracle at fixed Philox noise.

Tolerances: FP64 1e-10 relative to the largest block sum (rounding order
only); FP32 1e-5 (two-time) and 2e-3 relative on the gradients (each step's
reverse contraction rounds the cotangent to FP32, accumulated over the
window, the bound of the N = 32 FP32 test).
"""
import numpy as np
import pytest

from oracle import grad as ograd
from oracle import observables as oobs
from oracle import pump as opump
from oracle import twa as otwa

pytestmark = pytest.mark.gpu

KEYS = ("d_SpSm_dw", "d_SpSm_dalpha", "d_g2_dw", "d_g2_dalpha")


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


TWO_TIME_CASES = [
    # (precision, tile, N, B, tolerance)
    ("fp64", 1, 100, 40, 1e-10),
    ("fp64", 2, 130, 70, 1e-10),
    ("fp64", 3, 130, 70, 1e-10),
    ("fp32", 2, 300, 70, 1e-5),
    ("fp32", 7, 650, 130, 1e-5),
    ("fp32", 8, 650, 130, 1e-5),
    ("fp32", 7, 1000, 64, 1e-5),
    ("fp32", 1, 100, 40, 1e-5),
    # split BF16: 1e-4, the bound of its forward parity tests
    ("bf16x3", 2, 300, 70, 1e-4),
    ("bf16x3", 7, 650, 130, 1e-4),
]


@pytest.mark.parametrize("prec,cfg,N,B,tol", TWO_TIME_CASES)
def test_two_time_on_tile(twa, prec, cfg, N, B, tol):
    w, alpha, seed = 2.0, 1.0, 21
    dt, T, burn, L, stride = 0.02 / N, 120, 60, 7, 10
    p = twa.build_pump(N, w, alpha)
    print("two-time %s tile %d N=%d B=%d" % (prec, cfg, N, B), flush=True)
    r = twa.run(p, B, dt, T, seed=seed, precision=prec, tile_config=cfg, burnin=burn, n_lags=L, lag_stride=stride,
                want_lags=True, want_traj=True)
    assert r.obs["tile_config"] == cfg
    ref = otwa.run(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=seed, burnin=burn,
                                  n_lags=L, lag_stride=stride), opump.build_pump(N, w, alpha))
    corr = (r.corr_blocks[..., 0] + 1j * r.corr_blocks[..., 1]).T        # (J, L)
    chi = r.chi_blocks.transpose(1, 2, 0)                                # (J, 4, L)
    ec = np.max(np.abs(corr - ref.corr_blocks)) / np.abs(ref.corr_blocks).max()
    ex = np.max(np.abs(chi - ref.chi_blocks)) / np.abs(ref.chi_blocks).max()
    print("  corr rel %.2e chi rel %.2e" % (ec, ex))
    assert ec < tol and ex < tol, (ec, ex)
    # the response copies are not trivially zero or identical to the seed
    assert np.abs(ref.chi_blocks[:, :, -1]).max() > 0
    csym, chiv, c = oobs.two_time(ref.corr_blocks, ref.chi_blocks, B)
    om, S = oobs.spectrum(c, stride * dt)
    lw = oobs.fwhm(om, S)
    if np.isfinite(lw):
        assert abs(r.obs["linewidth"] - lw) < 1e3 * tol * abs(lw)


ADJOINT_CASES = [
    ("fp64", 2, 130, 40, 1e-8),
    ("fp64", 3, 130, 40, 1e-8),
    ("fp32", 2, 300, 64, 2e-3),
    ("fp32", 7, 650, 130, 2e-3),
    # split BF16: operands to 2^-17 (128x FP32's rounding) under the FP32 bound
    ("bf16x3", 2, 300, 64, 2e-3),
    ("bf16x3", 7, 650, 130, 2e-3),
]


@pytest.mark.parametrize("prec,cfg,N,B,tol", ADJOINT_CASES)
def test_adjoint_on_tile(twa, prec, cfg, N, B, tol):
    w, alpha, seed = 2.0, 1.0, 13
    dt, T, burn = 0.05 / N, 120, 60
    p = twa.build_pump(N, w, alpha)
    print("adjoint %s tile %d N=%d B=%d" % (prec, cfg, N, B), flush=True)
    obs, g = twa.adjoint(p, B, dt, T, seed=seed, ckpt_every=37, precision=prec, burnin=burn, tile_config=cfg)
    assert obs["tile_config"] == cfg
    ref = ograd.pathwise_gradients(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T,
                                                  seed=seed, burnin=burn))
    otol = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}[prec]
    for k in ("SpSm", "g2", "Sz"):
        assert abs(obs[k] - ref[k]) <= otol * max(1.0, abs(ref[k])), (k, obs[k], ref[k])
    for k in KEYS:
        err = abs(g[k] - ref[k])
        print("  %s gpu %.10g oracle %.10g rel %.2e" % (k, g[k], ref[k], err / max(abs(ref[k]), 1e-300)))
        atol = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-5}[prec] * max(1.0, abs(ref["SpSm"]))
        assert err <= tol * abs(ref[k]) + atol, (k, g[k], ref[k])
