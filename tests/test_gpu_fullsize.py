"""Parity at the full sizes of the paper's workloads, in the launch configuration
that bench.py times (default tile choice, graph replay), on outputs the FP64
oracle can compute one by one: trajectories are independent and their noise
counters carry the trajectory index, so the oracle integrates only the sampled
trajectories of the ensemble (``RunConfig.traj``).

Workloads (all synthetic, the method's own Philox stream):
  * N = 1e4, alpha = 1, w = ln N, 1024 trajectories, dt = 1e-4 (the headline
    workload; BF16 and FP32 contractions), sampled trajectories over 20 steps;
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


@pytest.fixture(scope="module")
def headline(twa):
    N, alpha, B, dt, T = 10000, 1.0, 1024, 1e-4, 20
    w = math.log(N)
    idx = np.array([0, 1, 513, 1023])
    pump = twa.build_pump(N, w, alpha)
    ref = otwa.run(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=len(idx), dt=dt, n_steps=T, seed=0,
                                  traj=idx), opump.build_pump(N, w, alpha))
    return dict(N=N, alpha=alpha, B=B, dt=dt, T=T, w=w, idx=idx, pump=pump, ref=ref)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_headline_workload_sampled_trajectories(twa, headline, prec):
    h = headline
    r = twa.run(h["pump"], h["B"], h["dt"], h["T"], seed=0, precision=prec, want_final_state=True,
                want_traj=True)
    g = r.final_state[:, h["idx"], :]
    rel = _max_rel_traj(g, h["ref"].final_state)
    mom = r.traj_moments[h["idx"]]
    mrel = float(np.max(np.abs(mom - h["ref"].traj_moments) / np.abs(h["ref"].traj_moments).max(axis=0)))
    print("N=1e4 %s tile %d: state rel %.3e moments rel %.3e" % (prec, r.obs["tile_config"], rel, mrel))
    # FP32: rounding of the FP32 state and operands only (1e-5 as at the smaller
    # sizes).  BF16: each step's contracted field increment (|dt/2 W s| +
    # |sqrt(dt) F zeta| ~ 0.04 of a spin at this workload) carries at most 2 u
    # relative error (u = 2^-9 for both operands), accumulated over 20 steps
    # without cancellation: 20 * 0.04 * 2^-8 ~ 3e-3.
    tol = {"fp32": 1e-5, "bf16": 5e-3}[prec]
    assert rel < tol, rel
    assert mrel < tol, mrel


def test_fp64_workload_n16_all_trajectories_and_ensemble(twa):
    N, alpha, w, B, dt, T = 16, 1.0, 4.0, 512, 1e-3, 20000
    pump = twa.build_pump(N, w, alpha)
    r = twa.run(pump, B, dt, T, seed=0, precision="fp64", s0z=-1.0, want_final_state=True, want_traj=True)
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
    r = twa.run(pump, B, dt, T, seed=0, precision="fp32", want_final_state=True)
    ref = otwa.run(otwa.RunConfig(n_spin=N, w=w, alpha=alpha, n_traj=len(idx), dt=dt, n_steps=T, seed=0,
                                  traj=idx), opump.build_pump(N, w, alpha))
    rel = _max_rel_traj(r.final_state[:, idx, :], ref.final_state)
    print("N=1000 fp32 1e3 steps tile %d: state rel %.3e" % (r.obs["tile_config"], rel))
    assert rel < 1e-5, rel
