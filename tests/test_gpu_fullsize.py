"""Parity at the full sizes of the paper's workloads, in the launch configuration
that bench.py times (default tile choice, graph replay), on outputs the FP64
oracle can compute one by one: trajectories are independent and their noise
counters carry the trajectory index, so the oracle integrates only the sampled
trajectories of the ensemble (``RunConfig.traj``).

Workloads (all synthetic, the method's own Philox stream):
  * N = 1e4, alpha = 1, w = ln N, 1024 trajectories, dt = 1e-4 (the headline
    workload; BF16, split BF16, FP32 and FP64 contractions, Heun and
    semi-implicit),
    sampled trajectories over 20 and 10^3 steps;
  * N = 16, alpha = 1, w = 4, 512 trajectories, dt = 1e-3, 2e4 steps, atoms
    initially down, FP64: every trajectory and the ensemble observables;
  * N = 1000, alpha = 1, w = 1, 4096 trajectories, dt = 1e-4, 1e3 steps,
    FP32: sampled trajectories.
"""
import math

import numpy as np
import pytest

from oracle import observables as oobs
from oracle import pump as opump
from oracle import twa as otwa

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def _max_rel_traj(g, o):
    """max over trajectories of |g_k - o_k|_2 / |o_k|_2 over the 3N components."""
    g = np.asarray(g).transpose(1, 0, 2).reshape(g.shape[1], -1)
    o = np.stack(o).transpose(1, 0, 2).reshape(g.shape[0], -1)
    return float(np.max(np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)))


HEADLINE = dict(N=10000, alpha=1.0, B=1024, dt=1e-4, w=math.log(10000))
HEADLINE_IDX = np.array([0, 1, 513, 1023])


@pytest.fixture(scope="module")
def headline(twa):
    """GPU pump of the headline workload and the oracle's sampled trajectories
    (computed on first use, per integrator and step count)."""
    h = HEADLINE
    gpump = twa.build_pump(h["N"], h["w"], h["alpha"])
    opump_ = opump.build_pump(h["N"], h["w"], h["alpha"])
    cache, errs = {}, {}

    def ref(integ, T):
        if (integ, T) not in cache:
            cfg = otwa.RunConfig(n_spin=h["N"], w=h["w"], alpha=h["alpha"], n_traj=len(HEADLINE_IDX), dt=h["dt"],
                                 n_steps=T, seed=0, traj=HEADLINE_IDX, integrator=integ)
            cache[(integ, T)] = otwa.run(cfg, opump_)
        return cache[(integ, T)]
    return dict(pump=gpump, ref=ref, errs=errs)


def _compare(twa, headline, integ, prec, T):
    if (integ, prec, T) in headline["errs"]:
        return headline["errs"][(integ, prec, T)]
    h = HEADLINE
    r = twa.run(headline["pump"], h["B"], h["dt"], T, seed=0, precision=prec, integrator=integ,
                want_final_state=True, want_traj=True, norm_tol=-1)
    ref = headline["ref"](integ, T)
    rel = _max_rel_traj(r.final_state[:, HEADLINE_IDX, :], ref.final_state)
    mom = r.traj_moments[HEADLINE_IDX]
    mrel = float(np.max(np.abs(mom - ref.traj_moments) / np.abs(ref.traj_moments).max(axis=0)))
    print("N=1e4 %s %s %d steps tile %d: state rel %.3e moments rel %.3e norm dev %.3g" % (
        integ, prec, T, r.obs["tile_config"], rel, mrel, r.obs["max_norm_dev"]))
    headline["errs"][(integ, prec, T)] = (rel, mrel)
    return rel, mrel


@pytest.mark.parametrize("integ,prec", [("heun", "fp32"), ("heun", "bf16"), ("sib", "bf16"), ("sib", "bf16x3")])
def test_headline_workload_sampled_trajectories(twa, headline, integ, prec):
    """20 steps of the headline workload, including the BF16 semi-implicit run
    the bench times and its equal-accuracy form in split BF16.  FP32:
    rounding of the FP32 state and operands only (1e-5).  BF16: each step's
    contracted field increment (|dt/2 W s| + |sqrt(dt) F zeta| ~ 0.04 of a
    spin at this workload) carries at most 2 u relative error (u = 2^-9 for
    both operands), accumulated over 20 steps without cancellation:
    20 * 0.04 * 2^-8 ~ 3e-3.  Split BF16: operands exact to 2^-17 and the
    dropped lo x lo product below 2^-18 give about 2^-16 per increment,
    20 * 0.04 * 2^-16 ~ 1.2e-5, on top of the FP32 state's 1e-5."""
    rel, mrel = _compare(twa, headline, integ, prec, 20)
    tol = {"fp32": 1e-5, "bf16": 5e-3, "bf16x3": 2.5e-5}[prec]
    assert rel < tol, rel
    assert mrel < tol, mrel


SIB_FP32_GROWTH = ("at step criterion 1.0 the semi-implicit map amplifies rounding faster than Heun's: measured "
                   "per-trajectory error 4.3e-7 (20 steps), 1.4e-6 (200), 2.9e-5 (1000) in FP32, and 1.1e-13 "
                   "against Heun's 2.6e-14 in FP64 at 1000 steps; the 1e-5 bound holds for Heun (4.6e-6)")


@pytest.mark.parametrize("integ,prec", [
    pytest.param("sib", "fp32", marks=pytest.mark.xfail(strict=True, reason=SIB_FP32_GROWTH)),
    ("sib", "fp64"), ("heun", "fp32"), ("heun", "fp64")])
def test_headline_workload_1e3_steps(twa, headline, integ, prec):
    """10^3 steps of the headline workload (step criterion max(Gamma N,
    lam_max) dt = 1.0) on sampled trajectories, in the launch configuration
    of the bench (1024 trajectories, default tiles: 320x256 in FP32, 128x128
    in FP64), FP32 at 1e-5 and FP64 at 1e-10 per trajectory."""
    rel, mrel = _compare(twa, headline, integ, prec, 1000)
    tol = {"fp32": 1e-5, "fp64": 1e-10}[prec]
    assert rel < tol, rel
    assert mrel < tol, mrel


@pytest.mark.parametrize("integ", ["sib", "heun"])
def test_headline_fp32_error_is_fp64_error_at_fp32_rounding(twa, headline, integ):
    """Over 10^3 steps at step criterion 1.0 the dynamics amplify rounding;
    the FP32 path's error against the oracle stays within the FP64 path's
    error scaled by the ratio of the unit round-offs (2^-24 / 2^-53), with a
    factor 2 for the randomness of rounding: the FP32 kernels add no error
    beyond binary32 arithmetic under the same amplification."""
    r32, _ = _compare(twa, headline, integ, "fp32", 1000)
    r64, _ = _compare(twa, headline, integ, "fp64", 1000)
    ratio = 2.0 ** -24 / 2.0 ** -53
    print("%s: fp32 %.3e, fp64 %.3e, fp64 x u32/u64 = %.3e" % (integ, r32, r64, r64 * ratio))
    assert r64 < 1e-10
    assert r32 < 2.0 * ratio * r64, (r32, r64)


def test_headline_split_bf16_error_is_fp64_error_at_its_rounding(twa, headline):
    """The equal-accuracy mode over 10^3 steps of the headline workload
    (semi-implicit): split BF16 represents each contracted increment to about
    2^-16 relative (operands to 2^-17, the dropped lo x lo product below
    2^-18), so under the same amplification of rounding its error against the
    oracle stays within the FP64 path's error scaled by 2^-16 / 2^-53, with a
    factor 2 as for FP32; it must also beat plain BF16 on the same steps."""
    r3, _ = _compare(twa, headline, "sib", "bf16x3", 1000)
    r64, _ = _compare(twa, headline, "sib", "fp64", 1000)
    r16, _ = _compare(twa, headline, "sib", "bf16", 1000)
    ratio = 2.0 ** -16 / 2.0 ** -53
    print("sib: bf16x3 %.3e, bf16 %.3e, fp64 %.3e, fp64 x u16/u64 = %.3e" % (r3, r16, r64, r64 * ratio))
    assert r3 < 2.0 * ratio * r64, (r3, r64)
    assert r3 < r16 / 10, (r3, r16)


def test_fp64_workload_n16_all_trajectories_and_ensemble(twa):
    N, alpha, w, B, dt, T = 16, 1.0, 4.0, 512, 1e-3, 20000
    pump = twa.build_pump(N, w, alpha)
    r = twa.run(pump, B, dt, T, seed=0, precision="fp64", s0z=-1.0, want_final_state=True, want_traj=True, norm_tol=-1)
    ref = otwa.run(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=T, seed=0, s0z=-1.0),
                   opump.build_pump(N, w, alpha))
    rel = _max_rel_traj(r.final_state, ref.final_state)
    mrel = float(np.max(np.abs(r.traj_moments - ref.traj_moments) / np.abs(ref.traj_moments).max(axis=0)))
    o = oobs.finalize(ref.traj_moments)
    orel = max(abs(r.obs[k] - o[k]) / max(1.0, abs(o[k])) for k in ("Sz", "SpSm", "g2", "SpSm_se", "g2_se"))
    print("N=16 fp64 2e4 steps: state rel %.3e moments rel %.3e observables rel %.3e" % (rel, mrel, orel))
    assert rel < 1e-10, rel
    assert mrel < 1e-10, mrel
    assert orel < 1e-10, orel


def test_fp32_workload_n1000_sampled_trajectories(twa):
    N, alpha, w, B, dt, T = 1000, 1.0, 1.0, 4096, 1e-4, 1000
    idx = np.array([0, 1, 2047, 4095])
    pump = twa.build_pump(N, w, alpha)
    r = twa.run(pump, B, dt, T, seed=0, precision="fp32", want_final_state=True, norm_tol=-1)
    ref = otwa.run(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=len(idx), dt=dt, n_steps=T, seed=0,
                                  traj=idx), opump.build_pump(N, w, alpha))
    rel = _max_rel_traj(r.final_state[:, idx, :], ref.final_state)
    print("N=1000 fp32 1e3 steps tile %d: state rel %.3e" % (r.obs["tile_config"], rel))
    assert rel < 1e-5, rel
