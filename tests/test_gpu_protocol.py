"""The paper's protocol and threshold quantities through the C ABI against the
oracle: the per-point protocol (step criterion, preparation time, window),
the fixed-noise threshold search (Newton steps with the forward-mode or
reverse-sweep pathwise derivative vs the oracle's bisection on its own runs),
and the g2_min scan."""
import numpy as np
import pytest

from oracle import protocol as oprot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


@pytest.mark.parametrize("N,w,alpha,fs", [(40, 2.0, 0.5, False), (40, 3.0, 1.5, False), (25, 0.7, 0.0, False),
                                          (30, 2.5, 1.0, True), (64, 1.2, 0.5, True)])
def test_protocol_matches_oracle(twa, N, w, alpha, fs):
    got = twa.protocol(twa.build_pump(N, w, alpha), 1.0, 0.04, finite_size=fs)
    ref = oprot.protocol(N, w, alpha, 1.0, 0.04, finite_size=fs)
    assert abs(got["dt"] - ref.dt) <= 1e-14 * ref.dt
    assert abs(got["tau_s"] - ref.tau_s) <= 1e-7 * ref.tau_s    # the oracle's eta is a truncated series
    assert got["tau"] == ref.tau
    assert got["n_prep"] == ref.n_prep and got["n_window"] == ref.n_window
    assert abs(got["wt"] - ref.wt) <= 1e-12 * ref.wt


N_T, ALPHA_T, B_T, DT_T, T_T, BURN_T, SEED_T = 10, 1.0, 256, 2e-3, 600, 300, 3


@pytest.mark.parametrize("objective,target,deriv", [("spsm_n", 1.0, "forward"), ("g2", 1.7, "forward"),
                                                    ("spsm_n", 1.0, "adjoint"), ("g2", 1.7, "adjoint")])
def test_threshold_matches_oracle_bisection(twa, objective, target, deriv):
    w, f, it = twa.find_threshold(N_T, ALPHA_T, B_T, DT_T, T_T, SEED_T, objective=objective, target=target,
                                  w_lo=1.0, w_hi=2.0, tol_w=1e-10, precision="fp64", burnin=BURN_T, norm_tol=-1,
                                  derivative=deriv)
    ref = oprot.bisect(lambda x: oprot.objective(N_T, x, ALPHA_T, B_T, DT_T, T_T, BURN_T, SEED_T, objective),
                       1.0, 2.0, target, tol=1e-10)
    print("threshold %s = %g (%s): GPU w %.12f (%d derivative evaluations, residual %.2e), oracle %.12f"
          % (objective, target, deriv, w, it, f, ref))
    assert abs(w - ref) < 1e-8 * ref
    assert abs(f) < 1e-8
    assert it <= 8


def test_threshold_fp32_converges_to_the_fp64_root(twa):
    w32, f, it = twa.find_threshold(N_T, ALPHA_T, B_T, DT_T, T_T, SEED_T, objective="spsm_n", target=1.0, w_lo=1.0,
                                    w_hi=2.0, tol_w=1e-6, precision="fp32", burnin=BURN_T, norm_tol=-1)
    w64, _, _ = twa.find_threshold(N_T, ALPHA_T, B_T, DT_T, T_T, SEED_T, objective="spsm_n", target=1.0, w_lo=1.0,
                                   w_hi=2.0, tol_w=1e-10, precision="fp64", burnin=BURN_T, norm_tol=-1)
    assert abs(f) < 1e-5 and it <= 10
    assert abs(w32 - w64) < 1e-4 * w64


def test_threshold_rejects_bracket_without_crossing(twa):
    with pytest.raises(twa.TWAError) as e:
        twa.find_threshold(N_T, ALPHA_T, 64, DT_T, 100, 0, objective="spsm_n", target=100.0, w_lo=1.0, w_hi=2.0,
                           precision="fp64", norm_tol=-1)
    assert e.value.code == -6


def test_g2_min_scan_matches_oracle(twa):
    N, alpha, B, wts = 8, 1.5, 128, [0.4, 0.7, 1.0]
    wt, g2, wmin, gmin = twa.g2_min(N, alpha, B, seed=2, n_points=3, wt_lo=0.4, wt_hi=1.0, precision="fp64", norm_tol=-1)
    ref = oprot.g2_scan(N, alpha, B, wts, seed=2)
    assert np.allclose(wt, wts, rtol=0, atol=1e-15)
    assert np.max(np.abs(g2 - ref) / ref) < 1e-9, (g2, ref)
    assert gmin == g2.min() and wmin == wt[int(np.argmin(g2))]
    assert int(np.argmin(g2)) == int(np.argmin(ref))


def test_protocol_rejects_bad_cfl(twa):
    with pytest.raises(twa.TWAError):
        twa.protocol(twa.build_pump(10, 1.0, 1.0), 1.0, 0.06)
