"""Normal-ordered observables, error bars and linewidth (oracle, FP64).

Test infrastructure only; see the package docstring.

* SM Sec. S1 step 6: <S+S-> = <S+S->_TWA + <S^z>_TWA / 2 and Eq. (S2):
  <S+S+S-S-> = <S+S+S-S->_TWA + 2 <S+ S^z S->_TWA - <S^z>_TWA / 3
               + <S^z S^z>_TWA / 2 - (4/3) <S+S->_TWA,
  with S^+ = (S^x + i S^y)/2 and S^mu = sum_i sigma^mu_i (Model section).
  The coefficients are implemented as printed.
* Main text (Observables and method): g2 = <S+S+S-S-> / <S+S->^2, a ratio of
  the ensemble- and time-averaged numerator and denominator.
* Error bars (the paper gives none): delete-one-block jackknife over
  contiguous trajectory blocks.
* Two-time (Eq. (S3) and the Kubo correction after it): the symmetric part is
  the classical product; the commutator part is
  kappa * i (chi_xx + chi_yy + i chi_yx - i chi_xy) with kappa = 1/4 as printed
  after Eq. (S3) (an alternative reading of the per-component formula gives
  1/16; both are available).  The symmetric part and the responses are
  pinned by tests; the weight kappa of their combination is fixed by the
  printed coefficient alone (parity unpinned for that one constant: no
  limit or closed form fixes it, and in the static limit the printed
  combination is not exact for any kappa).
* Spectrum S(omega) = 2 Re int dt e^{i omega t} <S+(t) S-(0)> over t >= 0;
  linewidth = full width at half maximum.
"""
from __future__ import annotations

import numpy as np

MOMENT_NAMES = ("T2", "T3", "T4", "Z", "ZZ")


def derived(m):
    """(Sz, SpSm, g2) from ensemble moments m = (T2, T3, T4, Z, ZZ)."""
    T2, T3, T4, Z, ZZ = m
    spsm = T2 + 0.5 * Z
    num = T4 + 2.0 * T3 - Z / 3.0 + 0.5 * ZZ - (4.0 / 3.0) * T2
    with np.errstate(divide="ignore", invalid="ignore"):
        return Z, spsm, num / (spsm * spsm)


def finalize(traj_moments: np.ndarray):
    """Ensemble observables and jackknife standard errors from per-trajectory
    time averages (n_traj, 5)."""
    B = traj_moments.shape[0]
    J = min(32, B)
    blk = (np.arange(B) * J) // B
    bsum = np.zeros((J, 5))
    np.add.at(bsum, blk, traj_moments)
    bcnt = np.bincount(blk, minlength=J).astype(np.float64)
    mean = bsum.sum(0) / B
    out = {n: float(v) for n, v in zip(MOMENT_NAMES, mean)}
    Sz, spsm, g2 = derived(mean)
    out.update(Sz=float(Sz), SpSm=float(spsm), g2=float(g2))
    if J >= 2:
        loo = (bsum.sum(0)[None, :] - bsum) / (B - bcnt)[:, None]
        vals = np.concatenate([loo, np.stack(derived(loo.T), axis=1)], axis=1)
        se = np.sqrt((J - 1) / J * ((vals - vals.mean(0)) ** 2).sum(0))
    else:
        se = np.full(8, np.nan)
    for name, s in zip(MOMENT_NAMES + ("Sz", "SpSm", "g2"), se):
        out[name + "_se"] = float(s)
    return out


def two_time(corr_blocks, chi_blocks, n_traj: int, kappa: float = 0.25):
    """Ensemble two-time correlation C(l) = C_sym(l) + kappa i (chi_xx + chi_yy
    + i chi_yx - i chi_xy), from block sums."""
    csym = corr_blocks.sum(0) / n_traj
    chi = chi_blocks.sum(0) / n_traj       # (4, L): xx, yx, xy, yy
    xx, yx, xy, yy = chi
    corr = csym + kappa * 1j * (xx + yy + 1j * yx - 1j * xy)
    return csym, chi, corr


def spectrum(corr: np.ndarray, tau: float, pad: int = 8):
    """S(omega) = 2 Re int_0^inf e^{i omega t} C(t) dt, trapezoid rule on the
    lag grid t_l = l tau, zero padded; returns (omega, S)."""
    L = corr.shape[0]
    n = pad * L
    c = np.zeros(n, dtype=np.complex128)
    c[:L] = corr
    c[0] *= 0.5                                   # trapezoid end points
    c[L - 1] *= 0.5
    # sum_l c_l e^{i omega_k t_l} with omega_k = 2 pi k / (n tau)
    s = n * np.fft.ifft(c)
    omega = 2.0 * np.pi * np.fft.fftfreq(n, d=tau)
    S = 2.0 * tau * s.real
    order = np.argsort(omega)
    return omega[order], S[order]


def fwhm(omega: np.ndarray, S: np.ndarray) -> float:
    """Full width at half maximum around the global peak, linear interpolation."""
    k = int(np.argmax(S))
    half = 0.5 * S[k]
    i = k
    while i > 0 and S[i] > half:
        i -= 1
    if S[i] > half:
        return float("nan")
    left = omega[i] + (half - S[i]) * (omega[i + 1] - omega[i]) / (S[i + 1] - S[i])
    j = k
    while j < len(S) - 1 and S[j] > half:
        j += 1
    if S[j] > half:
        return float("nan")
    right = omega[j - 1] + (half - S[j - 1]) * (omega[j] - omega[j - 1]) / (S[j] - S[j - 1])
    return float(right - left)
