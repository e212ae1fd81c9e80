"""Adjoint (reverse sweep with checkpointed recomputation) through the C ABI:
pathwise gradients against the FP64 oracle's tangent-linear gradient and
against central differences of the forward run at fixed noise."""
import numpy as np
import pytest

from oracle import grad as ograd
from oracle import observables as oobs
from oracle import twa as otwa

pytestmark = pytest.mark.gpu

KEYS = ("d_SpSm_dw", "d_SpSm_dalpha", "d_g2_dw", "d_g2_dalpha")


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def _close(a, b, rtol, atol=0.0):
    return abs(a - b) <= rtol * abs(b) + atol


@pytest.mark.parametrize("N,B,cfg,s0z", [(6, 24, 0, 1.0), (37, 20, 1, -1.0)])
def test_fp64_adjoint_matches_oracle_gradient(twa, N, B, cfg, s0z):
    w, alpha, dt, T, burn, seed = 2.0, 1.0, 2e-3, 240, 120, 7
    p = twa.build_pump(N, w, alpha)
    obs, g = twa.adjoint(p, B, dt, T, seed=seed, ckpt_every=37, precision="fp64", burnin=burn, s0z=s0z,
                         tile_config=cfg, norm_tol=-1)
    ref = ograd.pathwise_gradients(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T,
                                                  seed=seed, burnin=burn, s0z=s0z))
    for k in ("SpSm", "g2", "Sz"):
        assert _close(obs[k], ref[k], 1e-10, 1e-12), k
    for k in KEYS:
        assert _close(g[k], ref[k], 1e-8, 1e-10), (k, g[k], ref[k])


def test_adjoint_independent_of_checkpoint_spacing(twa):
    N, B, w, alpha, dt, T = 20, 16, 1.5, 0.7, 2e-3, 150
    p = twa.build_pump(N, w, alpha)
    _, g1 = twa.adjoint(p, B, dt, T, seed=3, ckpt_every=7, precision="fp64", norm_tol=-1)
    _, g2 = twa.adjoint(p, B, dt, T, seed=3, ckpt_every=150, precision="fp64", norm_tol=-1)
    _, g3 = twa.adjoint(p, B, dt, T, seed=3, ckpt_every=1000, precision="fp64", norm_tol=-1)
    for k in KEYS:
        assert g1[k] == g2[k] == g3[k]


def test_fp64_adjoint_matches_central_differences_of_the_gpu_run(twa):
    N, B, w, alpha, dt, T, h = 16, 32, 4.0, 1.0, 1e-3, 300, 1e-4
    p = twa.build_pump(N, w, alpha)
    _, g = twa.adjoint(p, B, dt, T, seed=0, precision="fp64", s0z=-1.0, norm_tol=-1)
    fd = {}
    for name, dw, da in (("w", h, 0.0), ("alpha", 0.0, h)):
        vals = []
        for sgn in (1, -1):
            q = twa.build_pump(N, w + sgn * dw, alpha + sgn * da)
            vals.append(twa.run(q, B, dt, T, seed=0, precision="fp64", s0z=-1.0, norm_tol=-1).obs)
        for o in ("SpSm", "g2"):
            fd["d_%s_d%s" % (o, name)] = (vals[0][o] - vals[1][o]) / (2 * h)
    for k in KEYS:
        assert _close(g[k], fd[k], 2e-5, 1e-8), (k, g[k], fd[k])


def test_fp32_adjoint_n32_against_oracle(twa):
    """The adjoint workload's oracle check size: N = 32, FP32 contraction."""
    N, B, w, alpha, dt, T = 32, 64, 2.0, 1.0, 1e-3, 300
    p = twa.build_pump(N, w, alpha)
    obs, g = twa.adjoint(p, B, dt, T, seed=0, precision="fp32", norm_tol=-1)
    ref = ograd.pathwise_gradients(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=0))
    for k in KEYS:
        assert _close(g[k], ref[k], 2e-3, 1e-6 * max(1.0, abs(ref["SpSm"]))), (k, g[k], ref[k])


def test_autograd_function(twa):
    import torch
    cfg = dict(N=12, n_traj=16, dt=2e-3, n_steps=120, seed=5, precision="fp64", ckpt_every=40, norm_tol=-1)
    w = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    spsm, g2 = twa.TWAObservables.apply(w, a, cfg)
    (spsm + 3.0 * g2).backward()
    p = twa.build_pump(12, 2.0, 0.8)
    _, g = twa.adjoint(p, 16, 2e-3, 120, seed=5, precision="fp64", ckpt_every=40, norm_tol=-1)
    assert abs(w.grad.item() - (g["d_SpSm_dw"] + 3 * g["d_g2_dw"])) < 1e-12 * max(1, abs(w.grad.item()))
    assert abs(a.grad.item() - (g["d_SpSm_dalpha"] + 3 * g["d_g2_dalpha"])) < 1e-12 * max(1, abs(a.grad.item()))


def test_adjoint_rejects_bad_arguments(twa):
    p = twa.build_pump(8, 1.0, 1.0)
    with pytest.raises(twa.TWAError):
        twa.adjoint(p, 8, 1e-3, 10, burnin=10, norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.adjoint(p, 8, 1e-3, 10, precision="bf16", norm_tol=-1)
    with pytest.raises(twa.TWAError):
        twa.adjoint(p, 8, 1e-3, 10, ckpt_every=0, norm_tol=-1)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_single_objective_sweep_equals_its_copy_of_the_joint_sweep(twa, prec):
    """Each objective is an independent copy of the reverse sweep: asking for one
    gives exactly that copy's gradients (the other entries are NaN)."""
    N, B, w, alpha, dt, T = 40, 48, 1.5, 0.8, 1e-3, 160
    p = twa.build_pump(N, w, alpha)
    _, both = twa.adjoint(p, B, dt, T, seed=3, ckpt_every=64, precision=prec, norm_tol=-1)
    for sel, keys in ((("g2",), ("d_g2_dw", "d_g2_dalpha")), (("SpSm",), ("d_SpSm_dw", "d_SpSm_dalpha"))):
        _, one = twa.adjoint(p, B, dt, T, seed=3, ckpt_every=64, precision=prec, objectives=sel, norm_tol=-1)
        for k in KEYS:
            if k in keys:
                assert one[k] == both[k], (sel, k)
            else:
                assert np.isnan(one[k])


def test_fp64_adjoint_n2000_matches_central_differences(twa):
    """The adjoint workload's pump (N = 2000, alpha = 1, w = 2, dt = 1e-4) on the
    path its run takes (default tiles, checkpointed reverse sweep) over 2048
    steps, FP64, against central differences of the forward run at fixed noise
    (h = 1e-4).  512 trajectories keep the FP64 checkpoint store small; the
    trajectories are independent, so the per-trajectory path is the
    workload's."""
    N, B, w, alpha, dt, T, h = 2000, 512, 2.0, 1.0, 1e-4, 2048, 1e-4
    p = twa.build_pump(N, w, alpha)
    obs, g = twa.adjoint(p, B, dt, T, seed=0, precision="fp64", ckpt_every=128, norm_tol=-1)
    fd = {}
    for name, dw, da in (("w", h, 0.0), ("alpha", 0.0, h)):
        vals = []
        for sgn in (1, -1):
            q = twa.build_pump(N, w + sgn * dw, alpha + sgn * da)
            vals.append(twa.run(q, B, dt, T, seed=0, precision="fp64", norm_tol=-1).obs)
            q.close()
        for o in ("SpSm", "g2"):
            fd["d_%s_d%s" % (o, name)] = (vals[0][o] - vals[1][o]) / (2 * h)
    print("N=2000 fp64 tile %d: max_norm_dev %.3g" % (obs["tile_config"], obs["max_norm_dev"]))
    for k in KEYS:
        print("  %s adjoint %.10g fd %.10g" % (k, g[k], fd[k]))
        assert _close(g[k], fd[k], 2e-5, 1e-8 * max(1.0, abs(obs["SpSm"]))), (k, g[k], fd[k])
