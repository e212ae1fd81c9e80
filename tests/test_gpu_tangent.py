"""Forward-mode pathwise derivatives in w (twa_tangent_w: one tangent-linear
copy with the field's own derivative Y/w - Q/(2w) as its source) through the
C ABI, against the FP64 oracle's tangent-linear gradient, against the
reverse sweep of twa_adjoint on the same runs, and central differences."""
import numpy as np
import pytest

from oracle import grad as ograd
from oracle import twa as otwa

pytestmark = pytest.mark.gpu

NAMES = {"d_SpSm_dw": "d_SpSm_dw", "d_g2_dw": "d_g2_dw", "d_Sz_dw": "d_Sz_dw"}


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


@pytest.mark.parametrize("prec,N,B,cfg,tol", [("fp64", 6, 24, 0, 1e-8), ("fp64", 37, 20, 1, 1e-8),
                                               ("fp64", 130, 40, 2, 1e-8), ("fp32", 32, 64, 0, 2e-3),
                                               ("fp32", 650, 130, 7, 2e-3), ("bf16x3", 130, 40, 2, 2e-3),
                                               ("bf16x3", 650, 130, 7, 2e-3)])
def test_tangent_matches_oracle_gradient(twa, prec, N, B, cfg, tol):
    """FP64 to rounding order; FP32 2e-3 (each step rounds the tangent's
    operands to FP32, accumulated over the window); split BF16 under the
    same bound: its operands carry 2^-17 instead of 2^-24, 128x FP32's
    rounding (measured at most 7e-6)."""
    w, alpha, seed, T = 2.0, 1.0, 7, 240
    dt = 0.1 / max(N, 20)
    burn = T // 2
    p = twa.build_pump(N, w, alpha)
    obs, g = twa.tangent_w(p, B, dt, T, seed=seed, precision=prec, tile_config=cfg, burnin=burn, s0z=-1.0,
                           norm_tol=-1)
    assert obs["tile_config"] == cfg
    ref = ograd.pathwise_gradients(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T,
                                                  seed=seed, burnin=burn, s0z=-1.0))
    otol = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-4}[prec]
    for k in ("SpSm", "g2", "Sz"):
        assert abs(obs[k] - ref[k]) <= otol * max(1.0, abs(ref[k])), (k, obs[k], ref[k])
    for k in NAMES:
        err = abs(g[k] - ref[k])
        print("%s N=%d tile %d %s: tangent %.12g oracle %.12g" % (prec, N, cfg, k, g[k], ref[k]))
        atol = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-5}[prec] * max(1.0, abs(ref["SpSm"]))
        assert err <= tol * abs(ref[k]) + atol, (k, g[k], ref[k])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x3", 1e-4)])
def test_tangent_equals_the_reverse_sweep(twa, prec, tol):
    """Forward and reverse mode give the same derivatives in w (the same
    runs: in FP64 only the summation order differs; in split BF16 each
    rounds its own operands to 2^-17, each within 1e-5 of the exact
    derivative)."""
    N, B, w, alpha, dt, T = 40, 48, 1.5, 0.8, 1e-3, 160
    p = twa.build_pump(N, w, alpha)
    _, ga = twa.adjoint(p, B, dt, T, seed=3, ckpt_every=64, precision=prec, norm_tol=-1)
    _, gt = twa.tangent_w(p, B, dt, T, seed=3, precision=prec, norm_tol=-1)
    for k in ("d_SpSm_dw", "d_g2_dw"):
        assert abs(ga[k] - gt[k]) <= tol * max(abs(ga[k]), 1e-3), (k, ga[k], gt[k])


def test_tangent_matches_central_differences(twa):
    N, B, w, alpha, dt, T, h = 300, 64, 2.0, 1.0, 2e-4, 400, 1e-4
    p = twa.build_pump(N, w, alpha)
    _, g = twa.tangent_w(p, B, dt, T, seed=1, precision="fp64", norm_tol=-1)
    vals = []
    for sgn in (1, -1):
        q = twa.build_pump(N, w + sgn * h, alpha)
        vals.append(twa.run(q, B, dt, T, seed=1, precision="fp64", norm_tol=-1).obs)
    for k, o in (("d_SpSm_dw", "SpSm"), ("d_g2_dw", "g2"), ("d_Sz_dw", "Sz")):
        fd = (vals[0][o] - vals[1][o]) / (2 * h)
        assert abs(g[k] - fd) <= 2e-5 * abs(fd) + 1e-8 * max(1.0, abs(vals[0]["SpSm"])), (k, g[k], fd)


def test_tangent_rejects_unsupported_runs(twa):
    p = twa.build_pump(20, 1.0, 1.0)
    with pytest.raises(twa.TWAError):
        twa.tangent_w(p, 8, 1e-3, 20, burnin=20)
    W = twa.build_pump(20, 1.0, 1.0).matrix("W")
    with pytest.raises(twa.TWAError):
        twa.tangent_w(twa.Pump(20, dense=W), 8, 1e-3, 20)
    with pytest.raises(twa.TWAError):
        twa.tangent_w(twa.build_pump(20, 0.0, 1.0), 8, 1e-3, 20)
