"""Planted mistakes in the oracle (CPU only).

Each case replaces one oracle function or constant with a plausible wrong
variant (a dropped term, a flipped sign, a slipped index, a wrong scale or
weight) for the duration of one test, and requires that at least one of the
named pins from tests/test_oracle_*.py then fails.  pytest's monkeypatch
restores the oracle afterwards, so nothing here changes what other tests see.
The variants below are written to differ from the oracle in exactly the one
planted place: ``test_unplanted_variants_equal_the_oracle`` checks that each
variant with no mistake planted reproduces the oracle bit for bit.
"""
import dataclasses
import os

import numpy as np
import pytest

from oracle import decay as odecay
from oracle import grad as ograd
from oracle import closed_forms, observables, philox, protocol, pump, toeplitz, twa
from tests import test_oracle_decay as tdecay
from tests import test_oracle_dynamics as dyn
from tests import test_oracle_exchange as texch
from tests import test_oracle_grad as tgrad
from tests import test_oracle_protocol as tproto
from tests import test_oracle_pump as tpump
from tests import test_oracle_rng as trng
from tests import test_oracle_sib as tsib
from tests import test_oracle_stationary as tstat
from tests import test_oracle_toeplitz as ttoep

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---- variants of the oracle's functions, each with one switchable mistake

def _increment(flip_pump=False, drop_collective=False, flip_z=False, y_field_from_x=False, flip_exchange=False):
    """Eq. (S1) increment, with the coherent exchange terms when W carries them."""
    def increment(state, W, gamma, dt, dxi, dchi):
        x, y, z = state
        Sx = x.sum(axis=1)[:, None]
        Sy = y.sum(axis=1)[:, None]
        c = 0.0 if drop_collective else 0.5 * gamma
        sgn = 0.5 if flip_pump else -0.5
        hx = (c * Sx + sgn * twa._matvec(W, x)) * dt + dxi[0][:, None] - dchi[0]
        hy = (c * Sy + sgn * twa._matvec(W, x if y_field_from_x else y)) * dt + dxi[1][:, None] - dchi[1]
        om = getattr(W, "omega", None)
        if om is not None:
            if flip_exchange:
                hx = hx - dt * (y @ om.T)
                hy = hy + dt * (x @ om.T)
            else:
                hx = hx + dt * (y @ om.T)
                hy = hy - dt * (x @ om.T)
        dz = (x * hx + y * hy) if flip_z else -(x * hx + y * hy)
        return z * hx, z * hy, dz, (hx, hy)
    return increment


def _noise_increments(drop_gamma=False, dt_for_sqrt_dt=False, same_pump_noise_xy=False):
    """Noise increments of one step for a dense pump."""
    def noise_increments(cfg, p, step):
        n, B = cfg.n_spin, cfg.n_traj
        gx, gy = philox.collective_noise(cfg.seed, step, B, cfg.point, cfg.traj)
        sg = np.sqrt(cfg.dt) if drop_gamma else np.sqrt(cfg.gamma * cfg.dt)
        sq = cfg.dt if dt_for_sqrt_dt else np.sqrt(cfg.dt)
        zx, zy = philox.pump_noise(cfg.seed, step, B, n, cfg.point, cfg.traj)
        if same_pump_noise_xy:
            zy = zx
        return (sg * gx, sg * gy), (sq * (zx @ p.F.T), sq * (zy @ p.F.T))
    return noise_increments


def _heun_step(corrector="trapezoid"):
    """Stochastic Heun step; the corrector is the trapezoid s + (D(s) + D(s~))/2."""
    def heun_step(state, W, gamma, dt, dxi, dchi):
        d1 = twa.increment(state, W, gamma, dt, dxi, dchi)
        pred = tuple(s + d for s, d in zip(state, d1[:3]))
        d2 = twa.increment(pred, W, gamma, dt, dxi, dchi)
        if corrector == "trapezoid":
            new = tuple(s + 0.5 * (a + b) for s, a, b in zip(state, d1[:3], d2[:3]))
        elif corrector == "sum":          # weights 1, 1 instead of 1/2, 1/2
            new = tuple(s + a + b for s, a, b in zip(state, d1[:3], d2[:3]))
        else:                             # the predictor alone (Euler)
            new = pred
        return new, (d1, pred, d2)
    return heun_step


def _sib_step(second_field_at="midpoint"):
    """Semi-implicit step; the second stage takes the field at (s_n + s~)/2."""
    def sib_step(state, W, gamma, dt, dxi, dchi):
        hx, hy = twa.fields(state, W, gamma, dt, dxi, dchi)
        pred = twa.midpoint_rotation(state, hx, hy)
        at = tuple(0.5 * (a + b) for a, b in zip(state, pred)) if second_field_at == "midpoint" else pred
        hx2, hy2 = twa.fields(at, W, gamma, dt, dxi, dchi)
        return twa.midpoint_rotation(state, hx2, hy2), pred
    return sib_step


def _derived(drop_half_z=False, c_t3=2.0, drop_z_third=False, c_zz=0.5, c_t2=4.0 / 3.0):
    """(Sz, <S+S->, g2) from the moments (SM Sec. S1 step 6, Eq. (S2))."""
    def derived(m):
        T2, T3, T4, Z, ZZ = m
        spsm = T2 if drop_half_z else T2 + 0.5 * Z
        zterm = 0.0 if drop_z_third else Z / 3.0
        num = T4 + c_t3 * T3 - zterm + c_zz * ZZ - c_t2 * T2
        with np.errstate(divide="ignore", invalid="ignore"):
            return Z, spsm, num / (spsm * spsm)
    return derived


def _moments(t2_scale=0.25):
    def moments(state):
        Sx, Sy, Sz = twa.collective_sums(*state)
        T2 = t2_scale * (Sx * Sx + Sy * Sy)
        return np.stack([T2, T2 * Sz, T2 * T2, Sz, Sz * Sz], axis=1)
    return moments


def _pump_matrix(flip_exponent=False):
    def pump_matrix(n_spin, w, alpha):
        i = np.arange(n_spin)
        d = np.abs(i[:, None] - i[None, :]).astype(np.float64)
        return w * (d + 1.0) ** alpha if flip_exponent else w / (d + 1.0) ** alpha
    return pump_matrix


def _box_muller(drop_two=False):
    def box_muller(a, b):
        a = np.asarray(a, dtype=np.uint64)
        b = np.asarray(b, dtype=np.uint64)
        u1 = ((a >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24
        u2 = (b >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
        r = np.sqrt(-np.log(u1)) if drop_two else np.sqrt(-2.0 * np.log(u1))
        return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)
    return box_muller


def _increment_tangent(drop_dz_h=False):
    """Directional derivative of the increment at fixed noise."""
    def increment_tangent(state, dstate, fields, W, gamma, dt):
        x, y, z = state
        dx, dy, dz = dstate
        hx, hy = fields
        dhx = (0.5 * gamma * dx.sum(axis=1)[:, None] - 0.5 * twa._matvec(W, dx)) * dt
        dhy = (0.5 * gamma * dy.sum(axis=1)[:, None] - 0.5 * twa._matvec(W, dy)) * dt
        if drop_dz_h:
            return z * dhx, z * dhy, -(dx * hx + x * dhx + dy * hy + y * dhy)
        return (dz * hx + z * dhx,
                dz * hy + z * dhy,
                -(dx * hx + x * dhx + dy * hy + y * dhy))
    return increment_tangent


def _incr_vjp(flip_collective=False, w_transposed=False):
    """Transpose of the increment's linearisation (reverse mode)."""
    def incr_vjp(state, mu, fields_dt, W, gamma, dt):
        x, y, z = state
        hx, hy = fields_dt
        ux, uy, uz = mu
        cx = -uz * hx
        cy = -uz * hy
        cz = ux * hx + uy * hy
        nx = ux * z - uz * x
        ny = uy * z - uz * y
        g = -0.5 * gamma if flip_collective else 0.5 * gamma
        Wm = W.T if w_transposed else W
        cx = cx + (g * nx.sum(axis=1)[:, None] - 0.5 * (nx @ Wm)) * dt
        cy = cy + (g * ny.sum(axis=1)[:, None] - 0.5 * (ny @ Wm)) * dt
        return cx, cy, cz
    return incr_vjp


def _first_column(mirror_off_by_one=False):
    def first_column(n_spin, w, alpha, M=None):
        M = toeplitz.embedding_size(n_spin) if M is None else M
        j = np.arange(M)
        d = np.minimum(j, M - 1 - j if mirror_off_by_one else M - j).astype(np.float64)
        return w / (1.0 + d) ** alpha
    return first_column


def _decay_derived(r_sign=-1.0):
    """(intensity, g2) of correlated emission from the nine quantities."""
    def derived(m):
        E2, E2E2, E2D, Q3, R, DD, U, V, D = m
        inten = E2 + 0.5 * D
        num = E2E2 + E2D + Q3 + r_sign * (R / 3.0) + 0.25 * (DD + U) - (4.0 / 3.0) * V
        with np.errstate(divide="ignore", invalid="ignore"):
            return inten, num / (inten * inten)
    return derived


def _spectrum(factor=2.0):
    def spectrum(corr, tau, pad=8):
        L = corr.shape[0]
        n = pad * L
        c = np.zeros(n, dtype=np.complex128)
        c[:L] = corr
        c[0] *= 0.5
        c[L - 1] *= 0.5
        s = n * np.fft.ifft(c)
        omega = 2.0 * np.pi * np.fft.fftfreq(n, d=tau)
        S = factor * tau * s.real
        order = np.argsort(omega)
        return omega[order], S[order]
    return spectrum


def _model_pump(drift_plus=False, noise_from_w=False):
    """Drift W - G and noise factor sqrt(W + G) of the correlated-decay step."""
    def model_pump(W, G):
        W = np.asarray(W, dtype=np.float64)
        G = np.asarray(G, dtype=np.float64)
        M = W + G
        lam, V = np.linalg.eigh(M)
        return pump.Pump(W.shape[0], float("nan"), float("nan"), W + G if drift_plus else W - G,
                         odecay.factor(W if noise_from_w else M), lam, V, float(lam[0]), float(lam[-1]))
    return model_pump


def _general_quantities(q3_slip=False):
    """The nine per-trajectory quantities of the correlated-emission estimator."""
    def general_quantities(state, G):
        x, y, z = state
        sp = 0.5 * (x + 1j * y)
        sm = 0.5 * (x - 1j * y)
        dg = np.diag(G)
        Gsm = sm @ G.T
        GTsp = sp @ G
        E2 = np.sum(sp * Gsm, axis=1).real
        D = z @ dg
        Q3 = np.sum(z * (Gsm if q3_slip else GTsp) * Gsm, axis=1).real
        R = z @ (dg * dg)
        U = np.sum(z * (z @ (G * G.T).T), axis=1)
        V = np.sum(dg * sp * Gsm, axis=1).real
        return np.stack([E2, E2 * E2, E2 * D, Q3, R, D * D, U, V, D], axis=1)
    return general_quantities


def _toeplitz_noise(drop_m=False):
    def noise(self, eps):
        scale = self.lam_plus if drop_m else self.lam_plus * self.M
        eta = np.fft.ifft(np.sqrt(scale)[None, :] * eps, axis=1)[:, :self.n_spin]
        return eta.real, eta.imag
    return noise


def _stationary_alpha0(flip_k=False):
    """Exact stationary TWA moments at alpha = 0 (the law of the rigidly
    rotating collective spin, exp(-k u) on u = cos theta)."""
    def stationary_alpha0(n_spin, gamma, w):
        vals, prob = closed_forms._rademacher_sum_law(n_spin)
        nodes, weights = np.polynomial.legendre.leggauss(200)
        acc = np.zeros(5)
        for X, pX in zip(vals, prob):
            for Y, pY in zip(vals, prob):
                R = np.sqrt(X * X + Y * Y + n_spin * n_spin)
                k = (gamma - w) * R / (gamma + w)
                E = closed_forms._u_moments(-k if flip_k else k, nodes, weights)
                s2 = 1.0 - nodes ** 2
                T2 = R ** 2 * E(s2) / 4.0
                T3 = R ** 3 * E(s2 * nodes) / 4.0
                T4 = R ** 4 * E(s2 ** 2) / 16.0
                Zm = R * E(nodes)
                ZZ = R ** 2 * E(nodes ** 2)
                acc += pX * pY * np.array([T2, T3, T4, Zm, ZZ])
        return acc
    return stationary_alpha0


def _dfactor(one_sided=False):
    """Derivative of the PSD square root along dW (Sylvester equation F X + X F = dW)."""
    def dfactor(p, dW):
        tol = 8.0 * p.n_spin * np.finfo(np.float64).eps * max(p.lam_max, 0.0)
        r = np.sqrt(np.where(p.lam > tol, p.lam, 0.0))
        B = p.V.T @ dW @ p.V
        den = 2.0 * r[:, None] + 0.0 * r[None, :] if one_sided else r[:, None] + r[None, :]
        Xp = np.where(den > 0, B / np.where(den > 0, den, 1.0), 0.0)
        X = p.V @ Xp @ p.V.T
        return 0.5 * (X + X.T)
    return dfactor


def _collective_noise(pump_tag=False):
    def collective_noise(seed, step, n_traj, point=0, traj=None):
        k0, k1 = philox.seed_key(seed)
        k = philox._traj_index(n_traj, traj)
        tag = philox.TAG_PUMP if pump_tag else philox.TAG_COLLECTIVE
        x0, x1, _, _ = philox.philox4x32_10(np.uint64(0), k, np.uint64(step), philox._tagword(tag, point), k0, k1)
        return philox.box_muller(x0, x1)
    return collective_noise


def _solve3(replace_row=False):
    """3 x 3 solves by Cramer's rule: column c of M replaced by r."""
    def solve3(M, r):
        def det(A):
            return (A[..., 0, 0] * (A[..., 1, 1] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 1])
                    - A[..., 0, 1] * (A[..., 1, 0] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 0])
                    + A[..., 0, 2] * (A[..., 1, 0] * A[..., 2, 1] - A[..., 1, 1] * A[..., 2, 0]))
        d = det(M)
        out = []
        for c in range(3):
            Mc = M.copy()
            if replace_row:
                Mc[..., c, :] = r
            else:
                Mc[..., :, c] = r
            out.append(det(Mc) / d)
        return out
    return solve3


def _t3_from_sz_squared(state):
    Sx, Sy, Sz = twa.collective_sums(*state)
    T2 = 0.25 * (Sx * Sx + Sy * Sy)
    return np.stack([T2, T2 * Sz * Sz, T2 * T2, Sz, Sz * Sz], axis=1)


def _finalize_round_robin_blocks(traj_moments):
    """The jackknife with trajectory k in block k mod J instead of the
    contiguous block floor(k J / B)."""
    B = traj_moments.shape[0]
    J = min(32, B)
    order = np.argsort(np.arange(B) % J, kind="stable")
    return _REAL_FINALIZE(traj_moments[order])


_REAL_PROTOCOL = protocol.protocol


def _protocol_tau_s_from_lam_min(N, w, alpha, gamma=1.0, cfl=0.04, finite_size=False, pump=None):
    pr = _REAL_PROTOCOL(N, w, alpha, gamma, cfl, finite_size, pump)
    if finite_size or alpha >= 1.0:
        return pr
    tau_s = 10.0 / pr.lam_min
    return dataclasses.replace(pr, tau_s=tau_s, n_prep=int(np.ceil(tau_s / pr.dt - 1e-9)))


def _protocol_without_gamma_n(N, w, alpha, gamma=1.0, cfl=0.04, finite_size=False, pump=None):
    pr = _REAL_PROTOCOL(N, w, alpha, gamma, cfl, finite_size, pump)
    dt = cfl / pr.lam_max
    return dataclasses.replace(pr, dt=dt, n_prep=int(np.ceil(pr.tau_s / dt - 1e-9)),
                               n_window=int(np.ceil(pr.tau / dt - 1e-9)))


def _quarter(omega, S):
    """Full width at a quarter of the maximum (the planted mistake)."""
    k = int(np.argmax(S))
    level = 0.25 * S[k]
    above = np.nonzero(S > level)[0]
    return float(omega[above[-1]] - omega[above[0]])


# ---- the planted mistakes and the pins that must notice each one

_REAL_BUILD_PUMP = pump.build_pump
_REAL_FINALIZE = observables.finalize
_REAL_DPUMP = pump.dpump_dalpha


def _build_pump_factor_is_w(n_spin, w, alpha):
    p = _REAL_BUILD_PUMP(n_spin, w, alpha)
    return dataclasses.replace(p, F=p.W.copy())


def _finalize_without_jackknife_factor(traj_moments):
    out = _REAL_FINALIZE(traj_moments)
    J = min(32, traj_moments.shape[0])
    for k in list(out):
        if k.endswith("_se"):
            out[k] *= np.sqrt(J / (J - 1.0))
    return out


CASES = {
    "pump drift with the wrong sign": (
        [(twa, "increment", _increment(flip_pump=True))],
        [lambda: dyn.test_sz_rate_at_t0_matches_lindblad(2, True), dyn.test_noiseless_correlated_pump_vs_dop853]),
    "collective drift Gamma S/2 dropped": (
        [(twa, "increment", _increment(drop_collective=True))],
        [dyn.test_noiseless_collective_decay_closed_form_second_order,
         lambda: dyn.test_sz_rate_at_t0_matches_lindblad(2, True)]),
    "ds^z with the wrong sign": (
        [(twa, "increment", _increment(flip_z=True))],
        [dyn.test_increment_orthogonal_to_spin]),
    "y field built from s^x (index slip)": (
        [(twa, "increment", _increment(y_field_from_x=True))],
        [dyn.test_noiseless_correlated_pump_vs_dop853]),
    "collective noise without Gamma": (
        [(twa, "noise_increments", _noise_increments(drop_gamma=True))],
        [tstat.test_noise_increments_follow_the_noise_law_of_eq_s1]),
    "pump noise scaled by dt instead of sqrt(dt)": (
        [(twa, "noise_increments", _noise_increments(dt_for_sqrt_dt=True))],
        [tstat.test_noise_increments_follow_the_noise_law_of_eq_s1]),
    "one pump noise for both x and y": (
        [(twa, "noise_increments", _noise_increments(same_pump_noise_xy=True))],
        [tstat.test_noise_increments_follow_the_noise_law_of_eq_s1]),
    "Heun corrector weights 1, 1": (
        [(twa, "heun_step", _heun_step("sum"))],
        [dyn.test_heun_norm_error_is_second_order_per_step,
         dyn.test_noiseless_collective_decay_closed_form_second_order]),
    "Heun corrector dropped (Euler)": (
        [(twa, "heun_step", _heun_step("euler"))],
        [dyn.test_noiseless_collective_decay_closed_form_second_order]),
    "midpoint rotation about +b": (
        [(twa, "midpoint_rotation", lambda st, hx, hy, f=twa.midpoint_rotation: f(st, -hx, -hy))],
        [tsib.test_midpoint_stage_is_the_rotation_about_minus_b,
         tsib.test_sib_noiseless_collective_decay_closed_form_second_order]),
    "semi-implicit second field at the predictor": (
        [(twa, "sib_step", _sib_step("predictor"))],
        [tsib.test_sib_noiseless_collective_decay_closed_form_second_order,
         tsib.test_sib_noiseless_correlated_pump_vs_dop853]),
    "<S+S-> without the S^z/2 ordering term": (
        [(observables, "derived", _derived(drop_half_z=True))],
        [lambda: dyn.test_initial_moments_exact_enumeration(2), dyn.test_sampled_initial_state,
         lambda: tstat.test_eq_s2_is_an_exact_operator_identity(3)]),
    "g2 numerator with -2 T3": (
        [(observables, "derived", _derived(c_t3=-2.0))],
        [lambda: tstat.test_alpha0_w_equals_gamma_g2_tends_to_paper_six_fifths(GOLDEN),
         lambda: tstat.test_eq_s2_is_an_exact_operator_identity(3)]),
    "g2 numerator without -S^z/3": (
        [(observables, "derived", _derived(drop_z_third=True))],
        [lambda: tstat.test_eq_s2_is_an_exact_operator_identity(3)]),
    "g2 numerator with ZZ instead of ZZ/2": (
        [(observables, "derived", _derived(c_zz=1.0))],
        [lambda: tstat.test_alpha0_w_equals_gamma_g2_tends_to_paper_six_fifths(GOLDEN),
         lambda: tstat.test_eq_s2_is_an_exact_operator_identity(3)]),
    "g2 numerator with -2/3 T2 instead of -4/3 T2": (
        [(observables, "derived", _derived(c_t2=2.0 / 3.0))],
        [lambda: tstat.test_alpha0_w_equals_gamma_g2_tends_to_paper_six_fifths(GOLDEN),
         lambda: tstat.test_eq_s2_is_an_exact_operator_identity(3)]),
    "T2 = |S|^2 / 2 instead of / 4": (
        [(twa, "moments", _moments(0.5))],
        [lambda: dyn.test_initial_moments_exact_enumeration(2)]),
    "Eq. (2) exponent with the wrong sign": (
        [(pump, "pump_matrix", _pump_matrix(flip_exponent=True))],
        [tpump.test_matrix_entries_eq2]),
    "noise factor F = W instead of its square root": (
        [(pump, "build_pump", _build_pump_factor_is_w), (twa, "build_pump", _build_pump_factor_is_w)],
        [lambda: tpump.test_factor_squares_to_w(33, 2.0, 0.5), tstat.test_pump_noise_covariance_equals_w]),
    "Box-Muller radius without the factor 2": (
        [(philox, "box_muller", _box_muller(drop_two=True))],
        [trng.test_box_muller_moments_and_ks]),
    "Philox Weyl increment off by one bit": (
        [(philox, "PHILOX_W1", np.uint64(0xBB67AE84))],
        [lambda: trng.test_philox_known_answers(GOLDEN)]),
    "jackknife without the (J-1)/J factor": (
        [(observables, "finalize", _finalize_without_jackknife_factor)],
        [tstat.test_jackknife_se_of_mean_matches_block_standard_error]),
    "tangent increment without dz h": (
        [(twa, "increment_tangent", _increment_tangent(drop_dz_h=True))],
        [tstat.test_response_fd_matches_tangent, tgrad.test_heun_vjp_is_the_transpose_of_the_tangent_step]),
    "reverse-mode collective term with the wrong sign": (
        [(ograd, "_incr_vjp", _incr_vjp(flip_collective=True))],
        [tgrad.test_heun_vjp_is_the_transpose_of_the_tangent_step]),
    "reverse-mode product with W instead of its transpose": (
        [(ograd, "_incr_vjp", _incr_vjp(w_transposed=True))],
        [tgrad.test_heun_vjp_is_the_transpose_of_the_tangent_step]),
    "circulant embedding mirrored at M - 1 - j": (
        [(toeplitz, "first_column", _first_column(mirror_off_by_one=True))],
        [lambda: ttoep.test_embedding_block_spectrum_and_drift(7, 1.0)]),
    "correlated-decay estimator with +R/3": (
        [(odecay, "derived", _decay_derived(r_sign=1.0))],
        [lambda: tdecay.test_estimator_is_an_exact_operator_identity(3, "random")]),
    "step criterion without Gamma N": (
        [(protocol, "protocol", _protocol_without_gamma_n)],
        [tproto.test_step_criterion_and_times]),
    "spectrum without the factor 2": (
        [(observables, "spectrum", _spectrum(factor=1.0))],
        [tstat.test_spectrum_of_exponential_has_fwhm_two_gamma]),
    "linewidth taken at a quarter of the maximum": (
        [(observables, "fwhm", _quarter)],
        [tstat.test_spectrum_of_exponential_has_fwhm_two_gamma]),
    "correlated-decay drift W + G instead of W - G": (
        [(odecay, "model_pump", _model_pump(drift_plus=True))],
        [tdecay.test_noiseless_correlated_decay_vs_dop853,
         lambda: tdecay.test_sz_rate_at_t0_matches_lindblad_with_correlated_decay(3, True, "free")]),
    "correlated-decay noise from W alone": (
        [(odecay, "model_pump", _model_pump(noise_from_w=True))],
        [tdecay.test_noise_covariance_is_pump_plus_decay]),
    "Q3 of the correlated-emission estimator with a slipped index": (
        [(odecay, "general_quantities", _general_quantities(q3_slip=True))],
        [tdecay.test_quantities_equal_brute_force_index_sums]),
    "coherent exchange field with the wrong sign": (
        [(twa, "increment", _increment(flip_exchange=True))],
        [texch.test_first_moments_at_t0_equal_the_heisenberg_rates_of_a_product_state,
         texch.test_noiseless_full_model_vs_dop853]),
    "circulant noise without the factor M": (
        [(toeplitz.ToeplitzPump, "noise", _toeplitz_noise(drop_m=True))],
        [ttoep.test_noise_covariance_is_the_pump]),
    "alpha = 0 stationary law with the wrong sign of k": (
        [(closed_forms, "stationary_alpha0", _stationary_alpha0(flip_k=True))],
        [tstat.test_alpha0_stationary_law_monte_carlo]),
    "square-root derivative with a one-sided denominator": (
        [(pump, "dfactor", _dfactor(one_sided=True))],
        [tpump.test_sylvester_factor_derivative]),
    "collective noise drawn on the pump stream": (
        [(philox, "collective_noise", _collective_noise(pump_tag=True))],
        [trng.test_streams_are_distinct_across_tags_points_steps]),
    "Cramer's rule with a row instead of a column replaced": (
        [(twa, "_solve3", _solve3(replace_row=True))],
        [tsib.test_midpoint_stage_is_the_rotation_about_minus_b]),
    "T3 built from (S^z)^2 instead of S^z": (
        [(twa, "moments", _t3_from_sz_squared)],
        [tstat.test_alpha0_stationary_law_monte_carlo]),
    "jackknife blocks round-robin instead of contiguous": (
        [(observables, "finalize", _finalize_round_robin_blocks)],
        [tstat.test_jackknife_se_of_mean_matches_block_standard_error]),
    "preparation time 10 / lambda_min also for alpha < 1": (
        [(protocol, "protocol", _protocol_tau_s_from_lam_min)],
        [tproto.test_step_criterion_and_times]),
    "d w_ij / d alpha with the wrong sign": (
        [(ograd, "dpump_dalpha", lambda n, w, a: -_REAL_DPUMP(n, w, a))],
        [tgrad.test_pathwise_gradient_matches_central_differences]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_planted_mistake_fails_a_pin(name, monkeypatch):
    patches, pins = CASES[name]
    for mod, attr, value in patches:
        monkeypatch.setattr(mod, attr, value)
    failed = []
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed.append(getattr(pin, "__name__", "pin"))
    assert failed, "no pin noticed the planted mistake: %s" % name


def test_unplanted_variants_equal_the_oracle():
    """The variants above with no mistake switched on are the oracle itself."""
    rng = np.random.default_rng(5)
    n, B, gamma, dt = 6, 4, 0.7, 1e-2
    p = pump.build_pump(n, 1.3, 0.9)
    st = tuple(rng.standard_normal((B, n)) for _ in range(3))
    dxi = (rng.standard_normal(B), rng.standard_normal(B))
    dchi = (rng.standard_normal((B, n)), rng.standard_normal((B, n)))
    for a, b in zip(_increment()(st, p.W, gamma, dt, dxi, dchi)[:3], twa.increment(st, p.W, gamma, dt, dxi, dchi)[:3]):
        assert np.array_equal(a, b)
    for a, b in zip(_heun_step()(st, p.W, gamma, dt, dxi, dchi)[0], twa.heun_step(st, p.W, gamma, dt, dxi, dchi)[0]):
        assert np.array_equal(a, b)
    for a, b in zip(_sib_step()(st, p.W, gamma, dt, dxi, dchi)[0], twa.sib_step(st, p.W, gamma, dt, dxi, dchi)[0]):
        assert np.array_equal(a, b)
    cfg = twa.RunConfig(n_spin=n, w=1.3, alpha=0.9, n_traj=B, dt=dt, n_steps=1, gamma=gamma, seed=3)
    for u, v in zip(_noise_increments()(cfg, p, 7), twa.noise_increments(cfg, p, 7)):
        for a, b in zip(u, v):
            assert np.array_equal(a, b)
    m = rng.standard_normal((5, 9))
    for a, b in zip(_derived()(m), observables.derived(m)):
        assert np.array_equal(a, b)
    assert np.array_equal(_moments()(st), twa.moments(st))
    assert np.array_equal(_pump_matrix()(9, 1.3, 0.9), pump.pump_matrix(9, 1.3, 0.9))
    Mq = rng.standard_normal((4, 3, 3)) + 3 * np.eye(3)
    rq = rng.standard_normal((4, 3))
    for a, b in zip(_solve3()(Mq, rq), twa._solve3(Mq, rq)):
        assert np.array_equal(a, b)
    dst = tuple(rng.standard_normal((B, n)) for _ in range(3))
    fl = twa.fields(st, p.W, gamma, dt, dxi, dchi)
    for a, b in zip(_increment_tangent()(st, dst, fl, p.W, gamma, dt), twa.increment_tangent(st, dst, fl, p.W, gamma, dt)):
        assert np.array_equal(a, b)
    Wn = rng.standard_normal((n, n))
    for a, b in zip(_incr_vjp()(st, dst, fl, Wn, gamma, dt), ograd._incr_vjp(st, dst, fl, Wn, gamma, dt)):
        assert np.array_equal(a, b)
    assert np.array_equal(_first_column()(130, 1.7, 0.8), toeplitz.first_column(130, 1.7, 0.8))
    q = rng.standard_normal((9, 5))
    for a, b in zip(_decay_derived()(q), odecay.derived(q)):
        assert np.array_equal(a, b)
    Gm = rng.standard_normal((n, n))
    Gm = Gm @ Gm.T / n
    a_, b_ = _model_pump()(p.W, Gm), odecay.model_pump(p.W, Gm)
    assert np.array_equal(a_.W, b_.W) and np.array_equal(a_.F, b_.F)
    assert np.array_equal(_general_quantities()(st, Gm), odecay.general_quantities(st, Gm))
    om = rng.standard_normal((n, n))
    om = om + om.T
    np.fill_diagonal(om, 0.0)
    ex = odecay.Exchange(p.W, om)
    for a, b in zip(_increment()(st, ex, gamma, dt, dxi, dchi)[:3], twa.increment(st, ex, gamma, dt, dxi, dchi)[:3]):
        assert np.array_equal(a, b)
    tp = toeplitz.ToeplitzPump(130, 1.7, 0.8)
    eps = tp.normals(3, 5, 4)
    for a, b in zip(_toeplitz_noise()(tp, eps), tp.noise(eps)):
        assert np.array_equal(a, b)
    assert np.array_equal(_stationary_alpha0()(6, 1.0, 0.5), closed_forms.stationary_alpha0(6, 1.0, 0.5))
    dW = rng.standard_normal((n, n))
    dW = dW + dW.T
    assert np.array_equal(_dfactor()(p, dW), pump.dfactor(p, dW))
    for a, b in zip(_collective_noise()(3, 7, 5), philox.collective_noise(3, 7, 5)):
        assert np.array_equal(a, b)
    corr = np.exp(-0.3 * np.arange(64)) * (1 + 0.1j)
    for a, b in zip(_spectrum()(corr, 0.05), observables.spectrum(corr, 0.05)):
        assert np.array_equal(a, b)
    words = philox.philox4x32_10(np.arange(64, dtype=np.uint64), 1, 2, 3, 4, 5)
    for a, b in zip(_box_muller()(words[0], words[1]), philox.box_muller(words[0], words[1])):
        assert np.array_equal(a, b)
