"""MI355X (gfx950) engine for dissipative Truncated-Wigner trajectories.

Thin Python binding of ``libtwa.so`` (C ABI declared in ``include/twa.h``):
argument marshalling only; every step of the time stepping runs in the
library's HIP kernels.  PyTorch is used only for device buffers and streams.
There is no CPU fallback: if the library is missing, importing the binding
raises, and without a GPU every compute call raises ``TWAError``.

Paper: Chelpanova, Stefanini, O'Keeffe, Marino, "Phase diagram of lasing
under correlated pump from GPU-accelerated Truncated Wigner dynamics";
equations of motion Eq. (S1), observables SM Sec. S1 and main text.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtwa.so")

TWA_OK, TWA_EINVAL, TWA_ENOMEM, TWA_EHIP, TWA_ENOTPSD, TWA_EUNSTABLE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "bf16x3": 4}
INTEGRATORS = {"heun": 0, "sib": 1}
PUMP_PATHS = {"dense": 0, "toeplitz": 1}


class TWAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("TWA error %d: %s" % (code, msg))
        self.code = code


class _Params(C.Structure):
    _fields_ = [("pump", C.c_void_p), ("gamma", C.c_double), ("s0z", C.c_double), ("burnin", C.c_int64),
                ("integrator", C.c_int32), ("precision", C.c_int32), ("n_lags", C.c_int64),
                ("lag_stride", C.c_int64), ("point", C.c_int32), ("tile_config", C.c_int32),
                ("stream", C.c_void_p), ("init_state", C.POINTER(C.c_double)), ("timing", C.c_int32),
                ("use_graph", C.c_int32), ("kappa", C.c_double), ("adjoint_objectives", C.c_int32),
                ("pump_path", C.c_int32), ("norm_tol", C.c_double)]


_OBS_DOUBLES1 = ["T2", "T3", "T4", "Z", "ZZ", "Sz", "SpSm", "g2",
                 "T2_se", "T3_se", "T4_se", "Z_se", "ZZ_se", "Sz_se", "SpSm_se", "g2_se"]


class _Obs(C.Structure):
    _fields_ = ([(n, C.c_double) for n in _OBS_DOUBLES1] +
                [("n_samples", C.c_int64), ("n_lags", C.c_int64), ("lag_stride", C.c_int64),
                 ("max_norm_dev", C.c_double), ("step_criterion", C.c_double), ("nan_flag", C.c_int32),
                 ("tile_config", C.c_int32), ("kernel_ms", C.c_double), ("stage1_ms", C.c_double),
                 ("stage1_launches", C.c_int64), ("stage2_ms", C.c_double), ("stage2_launches", C.c_int64),
                 ("gemm_flops", C.c_double), ("linewidth", C.c_double),
                 ("linewidth_sym", C.c_double), ("adjoint_fwd_ms", C.c_double), ("adjoint_bwd_ms", C.c_double),
                 ("I_gen", C.c_double), ("g2_gen", C.c_double), ("I_gen_se", C.c_double),
                 ("g2_gen_se", C.c_double)])


class _Outs(C.Structure):
    _fields_ = [("corr_blocks", C.POINTER(C.c_double)), ("chi_blocks", C.POINTER(C.c_double)),
                ("traj_moments", C.POINTER(C.c_double)), ("final_state", C.POINTER(C.c_double)),
                ("n_blocks", C.POINTER(C.c_int32)), ("traj_gen", C.POINTER(C.c_double))]


class _Point(C.Structure):
    _fields_ = [("N", C.c_int64), ("w", C.c_double), ("alpha", C.c_double), ("dt", C.c_double),
                ("seed", C.c_uint64)]


class _BatchOpts(C.Structure):
    _fields_ = [("n_traj", C.c_int64), ("n_steps", C.c_int64), ("burnin", C.c_int64), ("gamma", C.c_double),
                ("s0z", C.c_double), ("precision", C.c_int32), ("use_graph", C.c_int32),
                ("steps_per_graph", C.c_int32), ("tune_cache", C.c_char_p), ("stream", C.c_void_p),
                ("integrator", C.c_int32), ("norm_tol", C.c_double), ("n_lags", C.c_int64),
                ("lag_stride", C.c_int64), ("kappa", C.c_double), ("tile_config", C.c_int32),
                ("progress_every", C.c_int64), ("outputs", C.POINTER(_Outs))]


class _Protocol(C.Structure):
    _fields_ = [("dt", C.c_double), ("tau_s", C.c_double), ("tau", C.c_double), ("n_prep", C.c_int64),
                ("n_window", C.c_int64), ("wt", C.c_double), ("lam_min", C.c_double), ("lam_max", C.c_double)]


class _ThresholdOpts(C.Structure):
    _fields_ = [("objective", C.c_int32), ("target", C.c_double), ("w_lo", C.c_double), ("w_hi", C.c_double),
                ("tol_w", C.c_double), ("max_iter", C.c_int32), ("ckpt_every", C.c_int32),
                ("derivative", C.c_int32)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError("libtwa.so is not built (run __graft_entry__.build()); no CPU fallback exists")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.twa_last_error.restype = C.c_char_p
    lib.twa_version.restype = C.c_char_p
    lib.twa_build_pump.argtypes = [C.c_int64, C.c_double, C.c_double, C.POINTER(P)]
    lib.twa_build_pump_dense.argtypes = [C.c_int64, C.POINTER(C.c_double), C.POINTER(P)]
    lib.twa_build_pump_toeplitz.argtypes = [C.c_int64, C.c_double, C.c_double, C.POINTER(P)]
    lib.twa_build_model_dense.argtypes = [C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.POINTER(P)]
    lib.twa_pump_free.argtypes = [P]
    lib.twa_pump_free.restype = None
    lib.twa_pump_info.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.twa_pump_copy_matrix.argtypes = [P, C.c_int, C.POINTER(C.c_double)]
    lib.twa_params_default.argtypes = [C.POINTER(_Params)]
    lib.twa_params_default.restype = None
    lib.twa_run.argtypes = [C.POINTER(_Params), C.c_int64, C.c_double, C.c_int64, C.c_uint64, C.POINTER(_Obs),
                            C.POINTER(_Outs)]
    lib.twa_batch_opts_default.argtypes = [C.POINTER(_BatchOpts)]
    lib.twa_batch_opts_default.restype = None
    lib.twa_run_batch.argtypes = [C.POINTER(_Point), C.c_int, C.POINTER(_BatchOpts), C.POINTER(_Obs)]
    lib.twa_adjoint.argtypes = [C.POINTER(_Params), C.c_int64, C.c_double, C.c_int64, C.c_uint64, C.c_int32,
                                C.POINTER(_Obs), C.POINTER(C.c_double)]
    lib.twa_run_noalloc.argtypes = [C.POINTER(_Params), C.c_int64, C.c_double, C.c_int64, C.c_uint64,
                                    C.POINTER(_Obs)]
    lib.twa_tangent_w.argtypes = [C.POINTER(_Params), C.c_int64, C.c_double, C.c_int64, C.c_uint64,
                                  C.POINTER(_Obs), C.POINTER(C.c_double)]
    lib.twa_philox.argtypes = [P, C.c_int64, C.c_uint32, C.c_uint32, P, P]
    lib.twa_noise.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_int64, C.c_int64, C.c_int32, P, P, P]
    lib.twa_protocol.argtypes = [P, C.c_double, C.c_double, C.c_int32, C.POINTER(_Protocol)]
    lib.twa_threshold_opts_default.argtypes = [C.POINTER(_ThresholdOpts)]
    lib.twa_threshold_opts_default.restype = None
    lib.twa_find_threshold.argtypes = [C.c_int64, C.c_double, C.POINTER(_Params), C.c_int64, C.c_double, C.c_int64,
                                       C.c_uint64, C.POINTER(_ThresholdOpts), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.twa_g2_min.argtypes = [C.c_int64, C.c_double, C.POINTER(_Params), C.c_int64, C.c_uint64, C.c_int32,
                               C.c_double, C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    for name in ("twa_build_pump", "twa_build_pump_dense", "twa_build_pump_toeplitz", "twa_build_model_dense", "twa_pump_info", "twa_pump_copy_matrix", "twa_run",
                 "twa_run_batch", "twa_adjoint", "twa_tangent_w", "twa_run_noalloc", "twa_philox", "twa_noise", "twa_protocol", "twa_find_threshold",
                 "twa_g2_min"):
        getattr(lib, name).restype = C.c_int
    return lib


_lib = load_library()


def _check(rc: int):
    if rc != TWA_OK:
        raise TWAError(rc, _lib.twa_last_error().decode())


def version() -> str:
    return _lib.twa_version().decode()


def _stream_ptr(stream=None):
    if stream is not None:
        return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:   # pragma: no cover - torch missing
        pass
    return C.c_void_p(None)


class Pump:
    """Eq. (2) pump matrix, its channel decomposition and PSD noise factor
    (library-owned device memory, released on ``close``/garbage collection).
    With ``decay`` (and ``dense``): a model handle for correlated decay."""

    def __init__(self, N: int, w: float = None, alpha: float = None, dense: Optional[np.ndarray] = None,
                 decay: Optional[np.ndarray] = None, toeplitz_only: bool = False,
                 exchange: Optional[np.ndarray] = None):
        h = C.c_void_p()
        self.has_decay = decay is not None
        if toeplitz_only:
            _check(_lib.twa_build_pump_toeplitz(int(N), float(w), float(alpha), C.byref(h)))
        elif decay is not None:
            W = np.ascontiguousarray(dense, dtype=np.float64)
            G = np.ascontiguousarray(decay, dtype=np.float64)
            assert W.shape == (N, N) and G.shape == (N, N)
            O = None if exchange is None else np.ascontiguousarray(exchange, dtype=np.float64)
            assert O is None or O.shape == (N, N)
            _check(_lib.twa_build_model_dense(int(N), W.ctypes.data_as(C.POINTER(C.c_double)),
                                              G.ctypes.data_as(C.POINTER(C.c_double)),
                                              None if O is None else O.ctypes.data_as(C.POINTER(C.c_double)),
                                              C.byref(h)))
        elif dense is not None:
            W = np.ascontiguousarray(dense, dtype=np.float64)
            _check(_lib.twa_build_pump_dense(int(N), W.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)))
        else:
            _check(_lib.twa_build_pump(int(N), float(w), float(alpha), C.byref(h)))
        self._h = h
        self.N = int(N)
        self.w = w
        self.alpha = alpha
        n, lo, hi = C.c_int64(), C.c_double(), C.c_double()
        _check(_lib.twa_pump_info(self._h, C.byref(n), C.byref(lo), C.byref(hi)))
        self.lam_min, self.lam_max = lo.value, hi.value

    @property
    def handle(self):
        return self._h

    def matrix(self, which: str = "W") -> np.ndarray:
        """W (for a model handle: the drift matrix W - G), F (the noise factor)
        or G (model handles: the decay matrix)."""
        out = np.empty((self.N, self.N))
        _check(_lib.twa_pump_copy_matrix(self._h, {"W": 0, "F": 1, "G": 2, "Omega": 3}[which],
                                         out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.twa_pump_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_pump(N: int, w: float, alpha: float) -> Pump:
    return Pump(N, w, alpha)


def build_pump_toeplitz(N: int, w: float, alpha: float) -> Pump:
    """twa_build_pump_toeplitz: Eq. (2) for the Toeplitz fast path only."""
    return Pump(N, w, alpha, toeplitz_only=True)


def build_model(W: np.ndarray, decay: np.ndarray, exchange: Optional[np.ndarray] = None) -> Pump:
    """twa_build_model_dense: pump matrix W, correlated-decay matrix G and an
    optional coherent exchange Omega (symmetric, zero diagonal)."""
    W = np.asarray(W, dtype=np.float64)
    return Pump(W.shape[0], dense=W, decay=decay, exchange=exchange)


@dataclass
class RunResult:
    obs: dict
    traj_moments: Optional[np.ndarray] = None
    final_state: Optional[np.ndarray] = None
    corr_blocks: Optional[np.ndarray] = None
    chi_blocks: Optional[np.ndarray] = None
    n_blocks: int = 0
    status: int = 0
    traj_gen: Optional[np.ndarray] = None


def _obs_dict(o: _Obs) -> dict:
    return {name: getattr(o, name) for name, _ in _Obs._fields_}


def run(pump: Pump, n_traj: int, dt: float, n_steps: int, seed: int = 0, *, gamma: float = 1.0,
        s0z: float = 1.0, burnin: int = -1, precision: str = "fp32", n_lags: int = 0, lag_stride: int = 0,
        point: int = 0, tile_config: int = -1, init_state: Optional[np.ndarray] = None, timing: bool = False,
        use_graph: bool = True, kappa: float = 0.25, stream=None, want_traj: bool = False,
        want_final_state: bool = False, want_lags: bool = False, allow_unstable: bool = False,
        integrator: str = "heun", pump_path: str = "dense", norm_tol: float = 0.0) -> RunResult:
    """twa_run: n_traj trajectories of Eq. (S1), n_steps steps of size dt of the
    stochastic Heun ("heun") or semi-implicit midpoint ("sib") integrator; the
    pump applied by dense contractions ("dense") or through the circulant
    embedding of Eq. (2) ("toeplitz").  A run whose spin lengths drift by more
    than norm_tol (0: the library default 1e-2; < 0: no check) or that produces
    non-finite values returns TWA_EUNSTABLE: raised as TWAError unless
    allow_unstable (then ``status`` holds the code and the outputs are kept)."""
    p = _Params()
    _lib.twa_params_default(C.byref(p))
    p.pump = pump.handle
    p.pump_path = PUMP_PATHS[pump_path]
    p.integrator = INTEGRATORS[integrator]
    p.gamma, p.s0z, p.burnin = gamma, s0z, burnin
    p.precision = PRECISIONS[precision]
    p.n_lags, p.lag_stride, p.point, p.tile_config = n_lags, lag_stride, point, tile_config
    p.stream = _stream_ptr(stream)
    p.timing = 1 if timing else 0
    p.use_graph = 1 if use_graph else 0
    p.kappa = kappa
    p.norm_tol = norm_tol
    init = None
    if init_state is not None:
        init = np.ascontiguousarray(init_state, dtype=np.float64)
        assert init.shape == (3, n_traj, pump.N)
        p.init_state = init.ctypes.data_as(C.POINTER(C.c_double))
    o = _Obs()
    outs = _Outs()
    nb = C.c_int32(0)
    outs.n_blocks = C.pointer(nb)
    res = RunResult(obs={})
    J = min(32, n_traj)
    if want_traj:
        res.traj_moments = np.zeros((n_traj, 5))
        outs.traj_moments = res.traj_moments.ctypes.data_as(C.POINTER(C.c_double))
        if getattr(pump, "has_decay", False):
            res.traj_gen = np.zeros((n_traj, 9))
            outs.traj_gen = res.traj_gen.ctypes.data_as(C.POINTER(C.c_double))
    if want_final_state:
        res.final_state = np.zeros((3, n_traj, pump.N))
        outs.final_state = res.final_state.ctypes.data_as(C.POINTER(C.c_double))
    if want_lags and n_lags > 0:
        res.corr_blocks = np.zeros((n_lags, J, 2))
        res.chi_blocks = np.zeros((n_lags, J, 4))
        outs.corr_blocks = res.corr_blocks.ctypes.data_as(C.POINTER(C.c_double))
        outs.chi_blocks = res.chi_blocks.ctypes.data_as(C.POINTER(C.c_double))
    rc = _lib.twa_run(C.byref(p), int(n_traj), float(dt), int(n_steps), C.c_uint64(seed & (2 ** 64 - 1)),
                      C.byref(o), C.byref(outs))
    if not (rc == TWA_EUNSTABLE and allow_unstable):
        _check(rc)
    res.status = rc
    res.obs = _obs_dict(o)
    res.n_blocks = nb.value
    return res


def run_noalloc(pump: Pump, n_traj: int, dt: float, n_steps: int, seed: int = 0, *, gamma: float = 1.0,
                s0z: float = 1.0, burnin: int = -1, precision: str = "fp32", point: int = 0, tile_config: int = -1,
                integrator: str = "heun", stream=None, norm_tol: float = 0.0, allow_unstable: bool = False) -> dict:
    """twa_run_noalloc: the observables of twa_run for a run whose buffers fit
    the library's fixed device scratch array (no device allocation)."""
    p = _base_params(gamma, s0z, burnin, precision, point, tile_config, stream, norm_tol)
    p.pump = pump.handle
    p.integrator = INTEGRATORS[integrator]
    o = _Obs()
    rc = _lib.twa_run_noalloc(C.byref(p), int(n_traj), float(dt), int(n_steps), C.c_uint64(seed & (2 ** 64 - 1)),
                              C.byref(o))
    if not (rc == TWA_EUNSTABLE and allow_unstable):
        _check(rc)
    return _obs_dict(o)


def run_batch(points, n_traj: int, n_steps: int, *, burnin: int = -1, gamma: float = 1.0, s0z: float = 1.0,
              precision: str = "fp32", use_graph: bool = True, steps_per_graph: int = 16,
              tune_cache: Optional[str] = None, stream=None, integrator: str = "heun", norm_tol: float = 0.0,
              n_lags: int = 0, lag_stride: int = 0, kappa: float = 0.25, tile_config: int = -1, progress: int = 0,
              want_traj: bool = False, want_final_state: bool = False, want_lags: bool = False):
    """twa_run_batch: points is a sequence of (N, w, alpha, dt, seed); returns
    one observables dict per point (Philox point index = position), or, when
    per-trajectory arrays are requested (want_*), one RunResult per point.
    tile_config < 0 lets the library tune one tile configuration per N
    bucket; progress > 0 prints a line every that many steps."""
    n = len(points)
    pts = (_Point * n)()
    for i, (N, w, a, dt, seed) in enumerate(points):
        pts[i].N, pts[i].w, pts[i].alpha, pts[i].dt, pts[i].seed = int(N), float(w), float(a), float(dt), int(seed)
    o = _BatchOpts()
    _lib.twa_batch_opts_default(C.byref(o))
    o.n_traj, o.n_steps, o.burnin, o.gamma, o.s0z = n_traj, n_steps, burnin, gamma, s0z
    o.precision = PRECISIONS[precision]
    o.use_graph = 1 if use_graph else 0
    o.steps_per_graph = steps_per_graph
    o.tune_cache = tune_cache.encode() if tune_cache else None
    o.stream = _stream_ptr(stream)
    o.integrator = INTEGRATORS[integrator]
    o.norm_tol = norm_tol
    o.n_lags, o.lag_stride, o.kappa = n_lags, lag_stride, kappa
    o.tile_config = tile_config
    o.progress_every = progress
    arrays = want_traj or want_final_state or (want_lags and n_lags > 0)
    results = []
    if arrays:
        po = (_Outs * n)()
        J = min(32, n_traj)
        keep = []
        for i, (N, _, _, _, _) in enumerate(points):
            r = RunResult(obs={})
            nb = C.c_int32(0)
            keep.append(nb)
            po[i].n_blocks = C.pointer(nb)
            if want_traj:
                r.traj_moments = np.zeros((n_traj, 5))
                po[i].traj_moments = r.traj_moments.ctypes.data_as(C.POINTER(C.c_double))
            if want_final_state:
                r.final_state = np.zeros((3, n_traj, int(N)))
                po[i].final_state = r.final_state.ctypes.data_as(C.POINTER(C.c_double))
            if want_lags and n_lags > 0:
                r.corr_blocks = np.zeros((n_lags, J, 2))
                r.chi_blocks = np.zeros((n_lags, J, 4))
                po[i].corr_blocks = r.corr_blocks.ctypes.data_as(C.POINTER(C.c_double))
                po[i].chi_blocks = r.chi_blocks.ctypes.data_as(C.POINTER(C.c_double))
            results.append(r)
        o.outputs = po
    outs = (_Obs * n)()
    _check(_lib.twa_run_batch(pts, n, C.byref(o), outs))
    if not arrays:
        return [_obs_dict(x) for x in outs]
    for i, r in enumerate(results):
        r.obs = _obs_dict(outs[i])
        r.n_blocks = keep[i].value
    return results


GRAD_NAMES = ("d_SpSm_dw", "d_SpSm_dalpha", "d_g2_dw", "d_g2_dalpha")


def adjoint(pump: Pump, n_traj: int, dt: float, n_steps: int, seed: int = 0, *, ckpt_every: int = 256,
            gamma: float = 1.0, s0z: float = 1.0, burnin: int = -1, precision: str = "fp32", point: int = 0,
            tile_config: int = -1, stream=None, objectives=("SpSm", "g2"), norm_tol: float = 0.0,
            allow_unstable: bool = False):
    """twa_adjoint: observables of the forward run and the pathwise gradients
    d<S+S->/dw, d<S+S->/dalpha, dg2/dw, dg2/dalpha at fixed noise (those of
    objectives not requested are NaN; each objective costs one reverse copy).
    norm_tol and allow_unstable as in ``run``."""
    p = _Params()
    _lib.twa_params_default(C.byref(p))
    p.pump = pump.handle
    p.adjoint_objectives = (1 if "SpSm" in objectives else 0) | (2 if "g2" in objectives else 0)
    if p.adjoint_objectives == 0:
        raise ValueError("objectives must contain 'SpSm' and/or 'g2'")
    p.gamma, p.s0z, p.burnin = gamma, s0z, burnin
    p.precision = PRECISIONS[precision]
    p.point, p.tile_config = point, tile_config
    p.stream = _stream_ptr(stream)
    p.norm_tol = norm_tol
    o = _Obs()
    g = (C.c_double * 4)()
    rc = _lib.twa_adjoint(C.byref(p), int(n_traj), float(dt), int(n_steps), C.c_uint64(seed & (2 ** 64 - 1)),
                          int(ckpt_every), C.byref(o), g)
    if not (rc == TWA_EUNSTABLE and allow_unstable):
        _check(rc)
    return _obs_dict(o), dict(zip(GRAD_NAMES, list(g)))


TANGENT_NAMES = ("d_SpSm_dw", "d_g2_dw", "d_Sz_dw")


def tangent_w(pump: Pump, n_traj: int, dt: float, n_steps: int, seed: int = 0, *, gamma: float = 1.0,
              s0z: float = 1.0, burnin: int = -1, precision: str = "fp32", point: int = 0, tile_config: int = -1,
              stream=None, norm_tol: float = 0.0, allow_unstable: bool = False):
    """twa_tangent_w: observables of the forward run and the forward-mode
    pathwise derivatives d<S+S->/dw, dg2/dw, d<S^z>/dw at fixed noise."""
    p = _base_params(gamma, s0z, burnin, precision, point, tile_config, stream, norm_tol)
    p.pump = pump.handle
    o = _Obs()
    g = (C.c_double * 3)()
    rc = _lib.twa_tangent_w(C.byref(p), int(n_traj), float(dt), int(n_steps), C.c_uint64(seed & (2 ** 64 - 1)),
                            C.byref(o), g)
    if not (rc == TWA_EUNSTABLE and allow_unstable):
        _check(rc)
    return _obs_dict(o), dict(zip(TANGENT_NAMES, list(g)))


OBJECTIVES = {"g2": 0, "spsm_n": 1}
DERIVATIVES = {"forward": 0, "adjoint": 1}


def _base_params(gamma, s0z, burnin, precision, point, tile_config, stream, norm_tol=0.0):
    p = _Params()
    _lib.twa_params_default(C.byref(p))
    p.norm_tol = norm_tol
    p.gamma, p.s0z, p.burnin = gamma, s0z, burnin
    p.precision = PRECISIONS[precision]
    p.point, p.tile_config = point, tile_config
    p.stream = _stream_ptr(stream)
    return p


def protocol(pump: Pump, gamma: float = 1.0, cfl: float = 0.04, finite_size: bool = False) -> dict:
    """twa_protocol: time step, preparation time, window and step counts of the
    paper's protocol for one pump."""
    o = _Protocol()
    _check(_lib.twa_protocol(pump.handle, float(gamma), float(cfl), 1 if finite_size else 0, C.byref(o)))
    return {k: getattr(o, k) for k, _ in _Protocol._fields_}


def find_threshold(N: int, alpha: float, n_traj: int, dt: float, n_steps: int, seed: int = 0, *,
                   objective: str = "g2", target: float = 1.08, w_lo: float, w_hi: float, tol_w: float = 1e-6,
                   max_iter: int = 30, ckpt_every: int = 256, gamma: float = 1.0, s0z: float = 1.0,
                   burnin: int = -1, precision: str = "fp32", point: int = 0, tile_config: int = -1, stream=None,
                   norm_tol: float = 0.0, derivative: str = "forward"):
    """twa_find_threshold: the pump amplitude w where the fixed-noise objective
    ("g2" or "spsm_n" = <S+S->/N) equals target, by Newton steps with the
    forward-mode ("forward") or reverse-sweep ("adjoint") pathwise derivative;
    returns (w, objective - target, derivative evaluations).  norm_tol applies
    to every run of the search."""
    p = _base_params(gamma, s0z, burnin, precision, point, tile_config, stream, norm_tol)
    o = _ThresholdOpts()
    _lib.twa_threshold_opts_default(C.byref(o))
    o.objective, o.target, o.w_lo, o.w_hi = OBJECTIVES[objective], target, w_lo, w_hi
    o.derivative = DERIVATIVES[derivative]
    o.tol_w, o.max_iter, o.ckpt_every = tol_w, max_iter, ckpt_every
    w, f, it = C.c_double(), C.c_double(), C.c_int32()
    _check(_lib.twa_find_threshold(int(N), float(alpha), C.byref(p), int(n_traj), float(dt), int(n_steps),
                                   C.c_uint64(seed & (2 ** 64 - 1)), C.byref(o), C.byref(w), C.byref(f),
                                   C.byref(it)))
    return w.value, f.value, it.value


def g2_min(N: int, alpha: float, n_traj: int, seed: int = 0, *, n_points: int = 10, wt_lo: float = 0.1,
           wt_hi: float = 1.0, cfl: float = 0.04, finite_size: bool = False, gamma: float = 1.0,
           s0z: float = 1.0, precision: str = "fp32", point: int = 0, tile_config: int = -1, stream=None,
           norm_tol: float = 0.0):
    """twa_g2_min: g2 over n_points equally spaced w~ in [wt_lo, wt_hi], each point
    with its own protocol; returns (w~ array, g2 array, w~ of the minimum, g2_min)."""
    p = _base_params(gamma, s0z, -1, precision, point, tile_config, stream, norm_tol)
    wt = np.zeros(n_points)
    g2 = np.zeros(n_points)
    wmin, gmin = C.c_double(), C.c_double()
    _check(_lib.twa_g2_min(int(N), float(alpha), C.byref(p), int(n_traj), C.c_uint64(seed & (2 ** 64 - 1)),
                           int(n_points), float(wt_lo), float(wt_hi), float(cfl), 1 if finite_size else 0,
                           wt.ctypes.data_as(C.POINTER(C.c_double)), g2.ctypes.data_as(C.POINTER(C.c_double)),
                           C.byref(wmin), C.byref(gmin)))
    return wt, g2, wmin.value, gmin.value


def philox(ctr: np.ndarray, key0: int, key1: int) -> np.ndarray:
    """twa_philox on the device: ctr (n, 4) uint32 -> (n, 4) uint32."""
    import torch
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    n = c.shape[0]
    dc = torch.from_numpy(c.view(np.int32).copy()).cuda()
    do = torch.empty_like(dc)
    _check(_lib.twa_philox(C.c_void_p(dc.data_ptr()), n, key0, key1, C.c_void_p(do.data_ptr()), _stream_ptr()))
    return do.cpu().numpy().view(np.uint32)


def noise(seed: int, step: int, n_traj: int, N: int, point: int = 0, fp64: bool = True):
    """twa_noise: the step's Gaussians (zeta^x, zeta^y of shape (n_traj, N); g^x, g^y)."""
    import torch
    z = torch.empty((2, n_traj, N), dtype=torch.float64, device="cuda")
    g = torch.empty((2, n_traj), dtype=torch.float64, device="cuda")
    _check(_lib.twa_noise(C.c_uint64(seed), step, point, n_traj, N, 1 if fp64 else 0, C.c_void_p(z.data_ptr()),
                          C.c_void_p(g.data_ptr()), _stream_ptr()))
    z = z.cpu().numpy()
    g = g.cpu().numpy()
    return (z[0], z[1]), (g[0], g[1])


from .autograd import TWAObservables  # noqa: E402

__all__ = ["Pump", "build_pump", "run", "run_batch", "adjoint", "tangent_w", "philox", "noise", "TWAError", "version", "PRECISIONS",
           "LIB_PATH", "TWAObservables"]
