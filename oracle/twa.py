"""Dissipative TWA trajectories in FP64 (oracle; test infrastructure only).

Follows SM Sec. S1 of the paper step by step:

1. classical spins s_i = (s^x_i, s^y_i, s^z_i) replace the Pauli operators;
2. the stochastic equations of motion Eq. (S1), with collective noise xi^a
   (covariance Gamma, no site index: one noise per component shared by all
   spins) and pump noise chi^a_i (covariance w_ij);
3. discrete initial sampling s^{x,y} = +-1 with probability 1/2 and
   s^z = s0z (the paper uses +1, "all excited"; s0z = -1 prepares all atoms
   down);
5./6. trajectory averages of classical products, converted to normal order in
   ``oracle.observables``; equal-time observables are also averaged over the
   window (closing remark of SM Sec. S1);
and the two-time correlation (Eq. (S3) and the three-copy response that
follows it).  With ``RunConfig.decay`` the collective decay is replaced by a
correlated-decay matrix (``oracle.decay``) and the window also accumulates the
nine per-trajectory quantities of the correlated-emission estimator.  With
``RunConfig.toeplitz`` the pump is applied through its circulant embedding
(``oracle.toeplitz``), which also supplies the pump noise.

Readings where the paper is silent (listed with the others in the design
notes of the repository):

* Calculus / integrator: the paper integrates with a semi-implicit scheme and
  states that the equations preserve the spin length, which holds in the
  Stratonovich sense.  Integrators here: stochastic Heun (Euler predictor,
  trapezoidal corrector, the same noise increments in both stages; the
  default) and the semi-implicit midpoint scheme the paper cites (Mentink et
  al., 2010): each stage is the implicit midpoint rule with the field frozen,
  first at s_n, then at the midpoint of s_n and the first stage's result,
  which rotates every spin and keeps its length exactly.
* Discretisation of the noises over one step dt: xi^a dt -> sqrt(Gamma dt) g^a,
  chi^a dt -> sqrt(dt) (F zeta^a) with F the PSD square root of w_ij and g,
  zeta independent standard normals.
* Window: time averages over the states s_n, burnin < n <= n_steps.
* Two-time: single origin t0 = burnin * dt; lag l uses s_{burnin + l m} with
  stride m; the infinitesimal shifts of the response copies are propagated as
  tangent-linear copies (the eps -> 0 limit), or literally with a finite eps.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from . import decay as odecay
from . import philox
from . import toeplitz as otoe
from .pump import Pump, build_pump


@dataclass
class RunConfig:
    n_spin: int
    w: float
    alpha: float
    n_traj: int
    dt: float
    n_steps: int
    seed: int = 0
    gamma: float = 1.0
    s0z: float = 1.0
    burnin: Optional[int] = None      # default n_steps // 2
    n_lags: int = 0
    lag_stride: Optional[int] = None  # default max(1, (n_steps - burnin) // n_lags)
    point: int = 0
    noise: bool = True
    response_eps: Optional[float] = None   # None: tangent-linear response copies
    init_state: Optional[tuple] = None     # (x, y, z) arrays (n_traj, n_spin)
    integrator: str = "heun"               # "heun" or "sib" (semi-implicit midpoint)
    traj: Optional[np.ndarray] = None      # trajectory indices (n_traj,) of the noise counters;
                                           # None: 0 .. n_traj-1 (trajectories are independent,
                                           # so any subset of an ensemble can be integrated alone)
    decay: Optional[np.ndarray] = None     # (N, N) symmetric PSD correlated-decay matrix G; replaces
                                           # the collective decay (gamma unused), see oracle.decay
    exchange: Optional[np.ndarray] = None  # (N, N) symmetric zero-diagonal coherent exchange Omega
                                           # (oracle.decay.Exchange), Heun and semi-implicit only
    toeplitz: bool = False                 # apply Eq. (2) through its circulant embedding and draw
                                           # the pump noise from it (oracle.toeplitz)

    def resolved_burnin(self) -> int:
        return self.n_steps // 2 if self.burnin is None else int(self.burnin)

    def resolved_stride(self) -> int:
        if self.lag_stride is not None:
            return int(self.lag_stride)
        if self.n_lags <= 0:
            return 1
        return max(1, (self.n_steps - self.resolved_burnin()) // self.n_lags)


@dataclass
class RunResult:
    traj_moments: np.ndarray          # (n_traj, 5): time averages of T2, T3, T4, Z, ZZ
    n_samples: int
    final_state: tuple                # (x, y, z), each (n_traj, n_spin)
    corr_blocks: Optional[np.ndarray] = None   # (J, L) complex: block sums of the symmetric part
    chi_blocks: Optional[np.ndarray] = None    # (J, 4, L): block sums of chi_xx, chi_yx, chi_xy, chi_yy
    n_lags: int = 0
    lag_stride: int = 1
    max_norm_dev: float = 0.0
    extra: dict = field(default_factory=dict)


def initial_state(seed: int, n_traj: int, n_spin: int, s0z: float = 1.0, point: int = 0, traj=None):
    """Discrete sampling of SM Sec. S1 step 3."""
    sx, sy = philox.initial_signs(seed, n_traj, n_spin, point, traj)
    sz = np.full((n_traj, n_spin), float(s0z))
    return sx, sy, sz


def collective_sums(x, y, z):
    return x.sum(axis=1), y.sum(axis=1), z.sum(axis=1)


def _matvec(W, v):
    """sum_j W_ij v_j for every row of v: a dense matrix, or an operator with
    ``apply`` (the circulant embedding of Eq. (2))."""
    return W.apply(v) if hasattr(W, "apply") else v @ W.T


def increment(state, W, gamma, dt, dxi, dchi):
    """One-step increment of Eq. (S1) at a given state with given noise increments.

    h^a_i dt = (Gamma/2 S^a - 1/2 sum_j w_ij s^a_j) dt + dxi^a - dchi^a_i and
    ds^x_i = s^z_i h^x_i dt, ds^y_i = s^z_i h^y_i dt,
    ds^z_i = -(s^x_i h^x_i + s^y_i h^y_i) dt.
    ``dxi`` = (dxi^x, dxi^y), each (n_traj,); ``dchi`` = (dchi^x, dchi^y), each (n_traj, N).
    """
    x, y, z = state
    Sx = x.sum(axis=1)[:, None]
    Sy = y.sum(axis=1)[:, None]
    hx = (0.5 * gamma * Sx - 0.5 * _matvec(W, x)) * dt + dxi[0][:, None] - dchi[0]
    hy = (0.5 * gamma * Sy - 0.5 * _matvec(W, y)) * dt + dxi[1][:, None] - dchi[1]
    om = getattr(W, "omega", None)
    if om is not None:   # coherent exchange (oracle.decay.Exchange)
        hx = hx + dt * (y @ om.T)
        hy = hy - dt * (x @ om.T)
    return z * hx, z * hy, -(x * hx + y * hy), (hx, hy)


def increment_tangent(state, dstate, fields, W, gamma, dt):
    """Directional derivative of ``increment`` along ``dstate`` at fixed noise."""
    x, y, z = state
    dx, dy, dz = dstate
    hx, hy = fields
    if getattr(W, "omega", None) is not None:
        raise NotImplementedError("response copies are defined without coherent exchange")
    dhx = (0.5 * gamma * dx.sum(axis=1)[:, None] - 0.5 * _matvec(W, dx)) * dt
    dhy = (0.5 * gamma * dy.sum(axis=1)[:, None] - 0.5 * _matvec(W, dy)) * dt
    return (dz * hx + z * dhx,
            dz * hy + z * dhy,
            -(dx * hx + x * dhx + dy * hy + y * dhy))


def noise_increments(cfg: RunConfig, pump: Pump, step: int):
    """(dxi, dchi) of one step from the Philox stream."""
    n, B = cfg.n_spin, cfg.n_traj
    if not cfg.noise:
        z1 = np.zeros(B)
        zN = np.zeros((B, n))
        return (z1, z1), (zN, zN)
    gx, gy = philox.collective_noise(cfg.seed, step, B, cfg.point, cfg.traj)
    sg = np.sqrt(cfg.gamma * cfg.dt)
    sq = np.sqrt(cfg.dt)
    dxi = (sg * gx, sg * gy)
    if isinstance(pump, otoe.ToeplitzPump):
        ex, ey = pump.noise(pump.normals(cfg.seed, step, B, cfg.point, cfg.traj))
        return dxi, (sq * ex, sq * ey)
    zx, zy = philox.pump_noise(cfg.seed, step, B, n, cfg.point, cfg.traj)
    dchi = (sq * (zx @ pump.F.T), sq * (zy @ pump.F.T))
    return dxi, dchi


def heun_step(state, W, gamma, dt, dxi, dchi):
    """Stochastic Heun: predictor s~ = s + D(s), corrector s + (D(s) + D(s~))/2."""
    d1 = increment(state, W, gamma, dt, dxi, dchi)
    pred = tuple(s + d for s, d in zip(state, d1[:3]))
    d2 = increment(pred, W, gamma, dt, dxi, dchi)
    new = tuple(s + 0.5 * (a + b) for s, a, b in zip(state, d1[:3], d2[:3]))
    return new, (d1, pred, d2)


def fields(state, W, gamma, dt, dxi, dchi):
    """h^x_i dt and h^y_i dt of Eq. (S1) at a given state (as in ``increment``)."""
    return increment(state, W, gamma, dt, dxi, dchi)[3]


def _solve3(M, r):
    """Solve the 3 x 3 systems M s = r (M (..., 3, 3), r (..., 3)) by Cramer's
    rule: s_c = det(M with column c replaced by r) / det(M)."""
    def det(A):
        return (A[..., 0, 0] * (A[..., 1, 1] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 1])
                - A[..., 0, 1] * (A[..., 1, 0] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 0])
                + A[..., 0, 2] * (A[..., 1, 0] * A[..., 2, 1] - A[..., 1, 1] * A[..., 2, 0]))
    d = det(M)
    out = []
    for c in range(3):
        Mc = M.copy()
        Mc[..., :, c] = r
        out.append(det(Mc) / d)
    return out


def midpoint_rotation(state, hx, hy):
    """Solve s' = s + ((s + s') / 2) x b spin by spin, with b = (h^y dt, -h^x dt, 0)
    (so that s x b is the increment of Eq. (S1)): the implicit midpoint rule of
    ds = s x b with b held fixed, a 3 x 3 linear system per spin.  Writing
    [b] for the matrix of b x ., it reads (I + [b]/2) s' = (I - [b]/2) s,
    solved by Cramer's rule (det(I + [b]/2) = 1 + |b|^2/4 > 0)."""
    x, y, z = state
    bx, by = hy, -hx
    B, n = x.shape
    K = np.zeros((B, n, 3, 3))
    K[..., 0, 2] = by           # [b] = [[0, -bz, by], [bz, 0, -bx], [-by, bx, 0]], bz = 0
    K[..., 1, 2] = -bx
    K[..., 2, 0] = -by
    K[..., 2, 1] = bx
    eye = np.eye(3)
    s = np.stack([x, y, z], axis=-1)[..., None]
    rhs = ((eye - 0.5 * K) @ s)[..., 0]
    ox, oy, oz = _solve3(eye + 0.5 * K, rhs)
    return ox, oy, oz


def sib_step(state, W, gamma, dt, dxi, dchi):
    """Semi-implicit midpoint step (Mentink et al.): s~ = the midpoint rule with
    the field at s_n; s_{n+1} = the midpoint rule with the field at (s_n + s~)/2;
    the same noise increments in both stages."""
    hx, hy = fields(state, W, gamma, dt, dxi, dchi)
    pred = midpoint_rotation(state, hx, hy)
    mid = tuple(0.5 * (a + b) for a, b in zip(state, pred))
    hx2, hy2 = fields(mid, W, gamma, dt, dxi, dchi)
    return midpoint_rotation(state, hx2, hy2), pred


def step(cfg: RunConfig, state, W, dxi, dchi):
    """One step of the configured integrator."""
    if cfg.integrator == "heun":
        return heun_step(state, W, cfg.gamma, cfg.dt, dxi, dchi)[0]
    if cfg.integrator == "sib":
        return sib_step(state, W, cfg.gamma, cfg.dt, dxi, dchi)[0]
    raise ValueError("unknown integrator %r" % cfg.integrator)


def heun_step_tangent(state, dstate, W, gamma, dt, dxi, dchi, parts=None):
    """Tangent-linear Heun step (same noise) along ``dstate``."""
    if parts is None:
        _, parts = heun_step(state, W, gamma, dt, dxi, dchi)
    d1, pred, d2 = parts
    t1 = increment_tangent(state, dstate, d1[3], W, gamma, dt)
    dpred = tuple(a + b for a, b in zip(dstate, t1))
    t2 = increment_tangent(pred, dpred, d2[3], W, gamma, dt)
    return tuple(a + 0.5 * (b + c) for a, b, c in zip(dstate, t1, t2))


def moments(state):
    """T2 = |S^+|^2 = (S_x^2 + S_y^2)/4, T3 = T2 S_z, T4 = T2^2, Z = S_z, ZZ = S_z^2."""
    Sx, Sy, Sz = collective_sums(*state)
    T2 = 0.25 * (Sx * Sx + Sy * Sy)
    return np.stack([T2, T2 * Sz, T2 * T2, Sz, Sz * Sz], axis=1)


def n_blocks(n_traj: int) -> int:
    return min(32, n_traj)


def block_index(n_traj: int) -> np.ndarray:
    """Jackknife block of each trajectory: contiguous, near-equal blocks."""
    J = n_blocks(n_traj)
    return (np.arange(n_traj) * J) // n_traj


def run(cfg: RunConfig, pump: Optional[Pump] = None) -> RunResult:
    """Integrate all trajectories and accumulate the observables."""
    if pump is None:
        pump = build_pump(cfg.n_spin, cfg.w, cfg.alpha)
    if cfg.toeplitz:
        if cfg.decay is not None:
            raise ValueError("the circulant embedding applies to the pump of Eq. (2) only")
        pump = otoe.ToeplitzPump(cfg.n_spin, cfg.w, cfg.alpha)
    G = None
    if cfg.decay is not None:
        if cfg.n_lags > 0:
            raise NotImplementedError("two-time correlation of correlated emission is not defined here")
        G = np.asarray(cfg.decay, dtype=np.float64)
        pump = odecay.model_pump(pump.W, G)
        cfg = replace(cfg, gamma=0.0)    # the matrix replaces the collective terms
    W = pump if cfg.toeplitz else pump.W
    if cfg.exchange is not None:
        if cfg.toeplitz or cfg.n_lags > 0:
            raise NotImplementedError("coherent exchange: dense pump, no two-time response copies")
        W = odecay.Exchange(W, cfg.exchange)
    B, T = cfg.n_traj, cfg.n_steps
    burn = cfg.resolved_burnin()
    if cfg.init_state is not None:
        state = tuple(np.array(a, dtype=np.float64) for a in cfg.init_state)
    else:
        state = initial_state(cfg.seed, B, cfg.n_spin, cfg.s0z, cfg.point, cfg.traj)
    norm0 = state[0] ** 2 + state[1] ** 2 + state[2] ** 2

    acc = np.zeros((B, 5))
    gen_acc = np.zeros((B, 9)) if G is not None else None
    n_samples = 0
    L = int(cfg.n_lags)
    stride = cfg.resolved_stride()
    blk = block_index(B)
    J = n_blocks(B)
    corr_blocks = chi_blocks = None
    if L > 0:
        corr_blocks = np.zeros((J, L), dtype=np.complex128)
        chi_blocks = np.zeros((J, 4, L))
    eps = cfg.response_eps
    tan_x = tan_y = None
    Sm0 = None

    def lag_accumulate(l, st):
        Sx, Sy, _ = collective_sums(*st)
        sym = 0.25 * (Sx + 1j * Sy) * Sm0
        np.add.at(corr_blocks[:, l], blk, sym)
        if eps is None:
            cx = (tan_x[0].sum(1), tan_x[1].sum(1))
            cy = (tan_y[0].sum(1), tan_y[1].sum(1))
        else:
            cx = ((tan_x[0].sum(1) - Sx) / eps, (tan_x[1].sum(1) - Sy) / eps)
            cy = ((tan_y[0].sum(1) - Sx) / eps, (tan_y[1].sum(1) - Sy) / eps)
        for c, v in enumerate((cx[0], cx[1], cy[0], cy[1])):   # xx, yx, xy, yy
            np.add.at(chi_blocks[:, c, l], blk, v)

    def start_lags(st):
        nonlocal tan_x, tan_y, Sm0
        Sx, Sy, _ = collective_sums(*st)
        Sm0 = Sx - 1j * Sy
        one, zero = np.ones_like(st[0]), np.zeros_like(st[0])
        if eps is None:
            tan_x = (one, zero, zero.copy())
            tan_y = (zero.copy(), one.copy(), zero.copy())
        else:
            tan_x = (st[0] + eps, st[1].copy(), st[2].copy())
            tan_y = (st[0].copy(), st[1] + eps, st[2].copy())

    if L > 0 and cfg.integrator != "heun":
        raise NotImplementedError("two-time response copies are defined for the Heun integrator")
    if L > 0 and burn == 0:
        start_lags(state)
        lag_accumulate(0, state)
    for n in range(T):
        dxi, dchi = noise_increments(cfg, pump, n)
        if cfg.integrator == "heun":
            new, parts = heun_step(state, W, cfg.gamma, cfg.dt, dxi, dchi)
        else:
            new = step(cfg, state, W, dxi, dchi)
        if tan_x is not None:
            if eps is None:
                tan_x = heun_step_tangent(state, tan_x, W, cfg.gamma, cfg.dt, dxi, dchi, parts)
                tan_y = heun_step_tangent(state, tan_y, W, cfg.gamma, cfg.dt, dxi, dchi, parts)
            else:
                tan_x, _ = heun_step(tan_x, W, cfg.gamma, cfg.dt, dxi, dchi)
                tan_y, _ = heun_step(tan_y, W, cfg.gamma, cfg.dt, dxi, dchi)
        state = new
        k = n + 1
        if k > burn:
            acc += moments(state)
            if G is not None:
                gen_acc += odecay.general_quantities(state, G)
            n_samples += 1
        if L > 0:
            if k == burn:
                start_lags(state)
                lag_accumulate(0, state)
            elif k > burn and (k - burn) % stride == 0 and (k - burn) // stride < L:
                lag_accumulate((k - burn) // stride, state)
    traj = acc / max(n_samples, 1)
    norm1 = state[0] ** 2 + state[1] ** 2 + state[2] ** 2
    res = RunResult(traj_moments=traj, n_samples=n_samples, final_state=state,
                    corr_blocks=corr_blocks, chi_blocks=chi_blocks, n_lags=L,
                    lag_stride=stride, max_norm_dev=float(np.max(np.abs(norm1 - norm0))))
    if G is not None:
        res.extra["traj_gen"] = gen_acc / max(n_samples, 1)
    return res


def run_steps(state, pump: Pump, cfg: RunConfig, first_step: int, n_steps: int):
    """Advance a given state by ``n_steps`` steps of the configured integrator
    starting at step index ``first_step`` (noise counters follow the absolute
    step index)."""
    for n in range(first_step, first_step + n_steps):
        dxi, dchi = noise_increments(cfg, pump, n)
        state = step(cfg, state, pump.W, dxi, dchi)
    return state
