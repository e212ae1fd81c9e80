"""Statistical and closed-form pins of the oracle's noise, steady state and
two-time correlation."""
import numpy as np
import pytest

from oracle import closed_forms, lindblad, observables, philox, pump, twa


def test_pump_noise_covariance_equals_w():
    """<chi_i chi_j> dt = w_ij dt and <xi xi> dt = Gamma dt (Eq. (S1) noise law)."""
    n, w, alpha, B = 6, 1.7, 0.8, 4000
    p = pump.build_pump(n, w, alpha)
    samples, coll = [], []
    for step in range(60):
        zx, zy = philox.pump_noise(11, step, B, n)
        samples.append(zx @ p.F.T)
        samples.append(zy @ p.F.T)
        gx, gy = philox.collective_noise(11, step, B)
        coll.append(gx)
        coll.append(gy)
    X = np.concatenate(samples)
    M = X.shape[0]
    C = X.T @ X / M
    se = np.sqrt((np.outer(np.diag(p.W), np.diag(p.W)) + p.W ** 2) / M)
    assert np.all(np.abs(C - p.W) < 4.5 * se)
    g = np.concatenate(coll)
    assert abs(g.var() - 1.0) < 4.5 * np.sqrt(2.0 / g.size)


def test_noise_increments_follow_the_noise_law_of_eq_s1():
    """The increments the integrator is driven with, at Gamma != 1 and a small
    dt: <dxi^a dxi^b> = Gamma dt delta_ab, <dchi^a_i dchi^b_j> = w_ij dt delta_ab,
    and no correlation between the collective and the pump noise (Eq. (S1))."""
    n, B, gamma, dt, w, alpha = 5, 4000, 0.37, 2.5e-3, 1.7, 0.8
    p = pump.build_pump(n, w, alpha)
    cfg = twa.RunConfig(n_spin=n, w=w, alpha=alpha, n_traj=B, dt=dt, n_steps=1, gamma=gamma, seed=13)
    xi, chi = [], []
    for step in range(40):
        dxi, dchi = twa.noise_increments(cfg, p, step)
        xi.append(np.stack(dxi, axis=1))
        chi.append(np.concatenate(dchi, axis=1))
    X, C = np.concatenate(xi), np.concatenate(chi)
    M = X.shape[0]
    cx = X.T @ X / M                       # (2, 2)
    assert abs(cx[0, 0] / (gamma * dt) - 1) < 4.5 * np.sqrt(2.0 / M)
    assert abs(cx[1, 1] / (gamma * dt) - 1) < 4.5 * np.sqrt(2.0 / M)
    assert abs(cx[0, 1] / (gamma * dt)) < 4.5 / np.sqrt(M)
    cc = C.T @ C / M / dt                  # (2n, 2n): blocks xx, xy / yx, yy
    d = np.diag(p.W)
    se_same = np.sqrt((np.outer(d, d) + p.W ** 2) / M)
    se_cross = np.sqrt(np.outer(d, d) / M)
    assert np.all(np.abs(cc[:n, :n] - p.W) < 4.5 * se_same)
    assert np.all(np.abs(cc[n:, n:] - p.W) < 4.5 * se_same)
    assert np.all(np.abs(cc[:n, n:]) < 4.5 * se_cross)
    xc = X.T @ C / M / dt                  # (2, 2n)
    assert np.all(np.abs(xc) < 4.5 * np.sqrt(gamma * np.concatenate([d, d])[None, :] / M))


def _weyl(ops):
    """Fully symmetrised product of operators: the operator whose expectation
    the TWA average of the corresponding classical product is."""
    import itertools
    import math
    acc = np.zeros_like(ops[0])
    for perm in itertools.permutations(range(len(ops))):
        m = np.eye(ops[0].shape[0], dtype=ops[0].dtype)
        for j in perm:
            m = m @ ops[j]
        acc += m
    return acc / math.factorial(len(ops))


@pytest.mark.parametrize("n", [2, 3, 4])
def test_eq_s2_is_an_exact_operator_identity(n):
    """SM Sec. S1 step 6 and Eq. (S2): with the TWA moments T2 = |S+|^2,
    T3 = T2 S^z, T4 = T2^2, Z = S^z, ZZ = (S^z)^2 replaced by the exact
    expectations of the Weyl-ordered collective operators in a random mixed
    state, ``observables.derived`` returns the exact normal-ordered <S+S->
    and <S+S+S-S-> / <S+S->^2 (every coefficient of Eq. (S2) enters)."""
    ops = lindblad.operators(n)           # (sigma+, sigma-, sigma^z) per site
    Sp, Sm, Sz = sum(ops[0]), sum(ops[1]), sum(ops[2])
    Sx, Sy = Sp + Sm, -1j * (Sp - Sm)
    rng = np.random.default_rng(40 + n)
    d = 2 ** n
    R = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    rho = R @ R.conj().T
    rho /= np.trace(rho)

    def ev(op):
        return np.trace(rho @ op).real

    T2 = 0.25 * (ev(_weyl([Sx, Sx])) + ev(_weyl([Sy, Sy])))
    T3 = 0.25 * (ev(_weyl([Sx, Sx, Sz])) + ev(_weyl([Sy, Sy, Sz])))
    T4 = (ev(_weyl([Sx] * 4)) + 2 * ev(_weyl([Sx, Sx, Sy, Sy])) + ev(_weyl([Sy] * 4))) / 16.0
    Z, ZZ = ev(Sz), ev(Sz @ Sz)
    _, spsm, g2 = observables.derived(np.array([T2, T3, T4, Z, ZZ]))
    exact2 = ev(Sp @ Sm)
    exact4 = ev(Sp @ Sp @ Sm @ Sm)
    assert abs(spsm - exact2) < 1e-12 * max(1.0, abs(exact2))
    assert abs(g2 * spsm * spsm - exact4) < 1e-11 * max(1.0, abs(exact4))
    assert abs(T3) > 1e-3              # the state exercises every moment


def test_lindblad_collective_steady_state_is_detailed_balance():
    """Brute-force Eq. (1) at alpha = 0 from the all-up state relaxes to the
    detailed-balance populations quoted in the SM (collective pump)."""
    n, gamma, w = 4, 1.0, 0.6
    W = pump.pump_matrix(n, w, 0.0)
    rho = lindblad.steady_state(W, gamma, n, lindblad.product_state(n, True))
    ops = lindblad.operators(n)
    Sz = sum(ops[2])
    Sp = sum(ops[0])
    Sm = sum(ops[1])
    sz = lindblad.expect(rho, Sz).real
    spsm = lindblad.expect(rho, Sp @ Sm).real
    g2 = lindblad.expect(rho, Sp @ Sp @ Sm @ Sm).real / spsm ** 2
    ez, es, eg = closed_forms.dicke_alpha0(n, gamma, w)
    assert abs(sz - ez) < 1e-8 and abs(spsm - es) < 1e-8 and abs(g2 - eg) < 1e-8


def test_alpha0_stationary_law_monte_carlo():
    """alpha = 0, w = Gamma/2, N = 10: the Monte Carlo of Eq. (S1) approaches the
    exact stationary law of the rigidly rotating collective spin.  Heun's
    first-order length drift biases the moments by about 2 % at dt = 1e-3."""
    n, gamma, w = 10, 1.0, 0.5
    exact = closed_forms.stationary_alpha0(n, gamma, w)
    ez, es, eg = observables.derived(exact)
    assert abs(ez + 7.940) < 1e-3 and abs(es - 7.940) < 1e-3 and abs(eg - 1.519) < 1e-3
    cfg = twa.RunConfig(n_spin=n, w=w, alpha=0.0, n_traj=1024, dt=1e-3, n_steps=3000,
                        seed=2, burnin=1000)
    m = observables.finalize(twa.run(cfg).traj_moments)
    for key, ref in (("Sz", ez), ("SpSm", es), ("g2", eg)):
        tol = 4 * m[key + "_se"] + 0.04 * abs(ref)
        assert abs(m[key] - ref) < tol, (key, m[key], ref, m[key + "_se"])


def test_alpha0_w_equals_gamma_intensity_is_dicke():
    """At w = Gamma the law is uniform: <S+S-> = (N^2 + 2N)/6 (quantum Dicke value)."""
    n = 8
    exact = closed_forms.stationary_alpha0(n, 1.0, 1.0)
    assert abs(observables.derived(exact)[1] - (n * n + 2 * n) / 6.0) < 1e-10
    assert abs(closed_forms.dicke_alpha0(n, 1.0, 1.0)[1] - (n * n + 2 * n) / 6.0) < 1e-10
    cfg = twa.RunConfig(n_spin=n, w=1.0, alpha=0.0, n_traj=1024, dt=1e-3, n_steps=2500,
                        seed=5, burnin=1000)
    m = observables.finalize(twa.run(cfg).traj_moments)
    assert abs(m["SpSm"] - (n * n + 2 * n) / 6.0) < 4 * m["SpSm_se"] + 0.04 * (n * n + 2 * n) / 6.0
    assert abs(m["Sz"]) < 4 * m["Sz_se"] + 0.05


def test_two_time_alpha0_decays_at_gamma():
    """alpha = 0, w = Gamma: the drift vanishes, S diffuses rigidly and both the
    symmetric correlation and the response decay as exp(-Gamma t); the
    spectrum of the symmetric part has FWHM 2 Gamma (SM, collective pump)."""
    n = 6
    cfg = twa.RunConfig(n_spin=n, w=1.0, alpha=0.0, n_traj=768, dt=2e-3, n_steps=1500 + 1000,
                        seed=8, burnin=1500, n_lags=100, lag_stride=10)
    r = twa.run(cfg)
    csym, chi, _ = observables.two_time(r.corr_blocks, r.chi_blocks, cfg.n_traj)
    t = np.arange(100) * 10 * cfg.dt
    sel = t <= 1.0
    rate_c = -np.polyfit(t[sel], np.log(csym.real[sel]), 1)[0]
    rate_x = -np.polyfit(t[sel], np.log(chi[0][sel]), 1)[0]
    assert abs(rate_c - 1.0) < 0.15 and abs(rate_x - 1.0) < 0.1
    assert abs(chi[0][0] - n) < 1e-12 and abs(chi[3][0] - n) < 1e-12
    # symmetric part at lag 0 equals the intensity estimator at t0
    assert np.all(np.abs(csym.imag) < 0.2 * np.abs(csym.real[0]))


def test_response_fd_matches_tangent():
    base = dict(n_spin=5, w=2.0, alpha=1.0, n_traj=16, dt=1e-3, n_steps=200, seed=3,
                burnin=100, n_lags=10, lag_stride=10)
    rt = twa.run(twa.RunConfig(**base))
    rf = twa.run(twa.RunConfig(response_eps=1e-6, **base))
    assert np.allclose(rf.chi_blocks, rt.chi_blocks, rtol=0, atol=2e-4 * np.abs(rt.chi_blocks).max())
    assert np.array_equal(rf.corr_blocks, rt.corr_blocks)


def test_csym_lag0_equals_intensity_at_origin():
    cfg = twa.RunConfig(n_spin=4, w=1.0, alpha=0.5, n_traj=32, dt=1e-3, n_steps=20, seed=1,
                        burnin=20, n_lags=1)
    r = twa.run(cfg)
    t2 = twa.moments(r.final_state)[:, 0]
    assert np.isclose(r.corr_blocks.sum(), t2.sum(), rtol=1e-14)


def test_spectrum_of_exponential_has_fwhm_two_gamma():
    tau, L, g = 0.01, 4096, 0.7
    corr = np.exp(-g * tau * np.arange(L)).astype(np.complex128)
    om, S = observables.spectrum(corr, tau)
    assert abs(observables.fwhm(om, S) - 2 * g) < 0.01 * 2 * g
    # peak height 2/g of the Lorentzian 2 g / (g^2 + omega^2)
    assert abs(S.max() - 2.0 / g) < 0.01 * 2.0 / g


def test_jackknife_se_of_mean_matches_block_standard_error():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(256, 5))
    out = observables.finalize(x)
    bm = x.reshape(32, 8, 5).mean(1)
    for j, name in enumerate(observables.MOMENT_NAMES):
        assert np.isclose(out[name + "_se"], bm[:, j].std(ddof=1) / np.sqrt(32), rtol=1e-10)


def _paper_values(golden_dir):
    import os
    vals = {}
    for line in open(os.path.join(golden_dir, "paper_values.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_alpha0_w_equals_gamma_g2_tends_to_paper_six_fifths(golden_dir):
    """The exact stationary TWA law at alpha = 0, w = Gamma approaches the
    paper's printed g2 = 6/5 as N grows (1.2133, 1.2015, 1.2001 at N = 10, 40,
    200), from above and monotonically; a dropped moment or a wrong
    coefficient of Eq. (S2) moves the limit."""
    target = _paper_values(golden_dir)["g2_collective_pump_w_equals_gamma"]
    g = []
    for n in (10, 40, 200):
        g.append(observables.derived(closed_forms.stationary_alpha0(n, 1.0, 1.0))[2])
    assert abs(g[0] - 1.2133) < 1e-4 and abs(g[1] - 1.2015) < 1e-4
    assert abs(g[2] - target) < 2e-4
    assert g[0] > g[1] > g[2] > target


def test_alpha0_thermal_g2_tends_to_paper_two(golden_dir):
    """For w != Gamma the paper's collective-pump steady state is thermal,
    g2 -> 2 as N grows; the exact stationary TWA law reproduces that limit on
    both sides of w = Gamma, with an O(1/N) offset."""
    target = _paper_values(golden_dir)["g2_collective_pump_thermal"]
    for w in (0.25, 4.0):
        g = [observables.derived(closed_forms.stationary_alpha0(n, 1.0, w))[2] for n in (20, 80, 200)]
        errs = [abs(x - target) for x in g]
        assert errs[2] < 0.03, (w, g)
        assert errs[0] > errs[1] > errs[2], (w, g)
