/*
 * twa.h -- C ABI of the MI355X (gfx950) engine for the dissipative
 * Truncated-Wigner (TWA) trajectories of a chain of N two-level atoms under
 * collective cavity decay Gamma and the correlated incoherent pump
 * w_ij = w / (1 + |i - j|)^alpha.
 *
 * Paper: Chelpanova, Stefanini, O'Keeffe, Marino, "Phase diagram of lasing
 * under correlated pump from GPU-accelerated Truncated Wigner dynamics".
 *   - Model: Lindblad equation Eq. (1), pump profile Eq. (2), channel
 *     decomposition and normalised pump (text after Eq. (2) and Eq. (3)).
 *   - Method: SM Sec. S1 -- classical spins, the stochastic equations of
 *     motion Eq. (S1), discrete initial sampling, trajectory averages, the
 *     normal-ordering conversions (step 6 and Eq. (S2)), the two-time
 *     decomposition Eq. (S3) with the three-copy response, and time
 *     averaging over the window.
 *   - Observables and g2: main text, "Observables and method".
 *
 * Conventions for every entry point:
 *   - Return value 0 on success, a negative TWA_E* code on failure; no C++
 *     exception crosses this boundary.  twa_last_error() returns a
 *     thread-local message describing the last failure of the calling thread.
 *   - Pointers documented as "host" are ordinary CPU memory owned by the
 *     caller; pointers documented as "device" are HIP device memory owned by
 *     the caller.  Library-owned objects (twa_pump) are released with their
 *     free function.
 *   - `stream` arguments are hipStream_t passed as void*.  Every compute
 *     entry point is stream-ordered on that stream and returns after its
 *     results are on the host unless stated otherwise; with NULL it runs on a
 *     non-blocking stream of its own (twa_run_noalloc: on the null stream).
 *   - Host threads: every entry point that touches a device takes one
 *     process-wide lock for its whole duration, so calls from several host
 *     threads are safe and run one at a time.  The reason: releasing device
 *     memory (hipFree) synchronises the whole device, which invalidates a
 *     hipGraph capture that another thread has open.  Each call owns its
 *     buffers, pump handles are only read by runs, graphs are captured in
 *     thread-local mode on the call's own stream, and no call issues work on
 *     the null stream (twa_run_noalloc given NULL aside).  The lock does not
 *     extend to other code in the process: a library call that releases
 *     memory synchronises the device, so it must not overlap a hipGraph
 *     capture that another thread holds open outside the library.
 *   - All arithmetic of the time stepping runs in the library's HIP kernels
 *     for gfx950.  There is no CPU fallback: without a usable GPU every
 *     compute entry point returns TWA_EHIP.
 */
#ifndef TWA_H
#define TWA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TWA_API __attribute__((visibility("default")))

/* ---- status codes ---------------------------------------------------- */
#define TWA_OK          0
#define TWA_EINVAL     -1   /* an argument is out of range or inconsistent     */
#define TWA_ENOMEM     -2   /* device or host allocation failed                */
#define TWA_EHIP       -3   /* a HIP / rocSOLVER / rocBLAS call failed         */
#define TWA_ENOTPSD    -4   /* pump matrix has a negative eigenvalue below     */
                            /* -1e-10 * lambda_max (Eq. (2) is PSD; this flags */
                            /* a non-PSD dense matrix)                         */
#define TWA_EUNSTABLE  -5   /* NaN/Inf in the state or accumulators, or a spin */
                            /* length that drifted: max_norm_dev above the    */
                            /* run's norm_tol (Eq. (S1) keeps every |s_i|^2,  */
                            /* SM Sec. S1).  Outputs are still written so     */
                            /* they can be inspected                          */
#define TWA_ENOROOT    -6   /* threshold search: the objective does not cross  */
                            /* the target on the bracket, or no convergence    */

/* ---- precisions of the channel-mixing contraction ---------------------- */
#define TWA_PREC_FP64   0   /* FP64 state, FP64 MFMA contraction               */
#define TWA_PREC_FP32   1   /* FP32 state, FP32 MFMA contraction               */
#define TWA_PREC_BF16   2   /* FP32 state, BF16 MFMA inputs, FP32 accumulation */
#define TWA_PREC_FP16   3   /* FP32 state, FP16 MFMA inputs, FP32 accumulation */
#define TWA_PREC_BF16X3 4   /* FP32 state; each contraction operand split into   */
                            /* bf16 hi + lo (x = hi + lo + O(2^-17 |x|)) and the  */
                            /* product formed as Ahi Xhi + Ahi Xlo + Alo Xhi on   */
                            /* BF16 MFMA with FP32 accumulation (the split scheme */
                            /* of Henry, Tang and Heinecke 2019): near-FP32       */
                            /* accuracy at three BF16 contractions.  Runs (two-   */
                            /* time lags included), batches, twa_tangent_w and    */
                            /* twa_adjoint; dense pumps without decay matrix      */

/* tile_config reported when the fused small-N kernel integrated the run */
#define TWA_TILE_FUSED  99
/* tile_config reported when the Toeplitz fast path integrated the run */
#define TWA_TILE_TOEPLITZ 98

/* ---- how the pump of Eq. (2) is applied -------------------------------- */
#define TWA_PUMP_DENSE    0 /* MFMA contractions with W and its PSD square root F */
#define TWA_PUMP_TOEPLITZ 1 /* not in the paper: circulant embedding of the Toeplitz
                               matrix of Eq. (2) (first column c(min(j, M-j)),
                               c(d) = w/(1+d)^alpha, M = max(256, 2^ceil(log2(2N-2))),
                               PSD for this convex decreasing c); W s by FFT
                               products and the pump noise drawn from the
                               embedding, IDFT(sqrt(lam M) eps)[:N] with complex
                               normals eps from Philox tag 3 (eps_k and
                               eps_{k+M/2} from one call): equal in law to the
                               dense path, not pathwise.  Heun, FP64 (N <= 8193)
                               or FP32 (N <= 16385), a pump from twa_build_pump,
                               no two-time lags.  O(M log M) per trajectory-step */

/* ---- integrators ------------------------------------------------------ */
#define TWA_INT_HEUN    0   /* stochastic Heun, Stratonovich reading of Eq. (S1) */
#define TWA_INT_SIB     1   /* semi-implicit midpoint scheme (the spin-length-preserving
                               integrator the paper cites): each of the two stages is the
                               implicit midpoint rule with the field frozen, first at s_n,
                               then at the midpoint of s_n and the first stage's result;
                               not available with n_lags > 0 or in twa_adjoint */

/* ======================================================================
 * Pump: Eq. (2) and its channel decomposition.
 * ====================================================================== */
typedef struct twa_pump twa_pump;   /* opaque, library-owned */

/*
 * twa_build_pump -- build w_ij = w / (|i-j| + 1)^alpha (Eq. (2), open chain,
 * i, j = 0..N-1) in FP64 on the device, diagonalise it (the channel rates of
 * the text after Eq. (2)), and form the noise factor F, the symmetric
 * positive-semidefinite square root V diag(sqrt(lambda+)) V^T, where lambda+
 * zeroes eigenvalues below 8 N eps lambda_max (round-off of the rank-one
 * alpha = 0 case).  F colours the pump noise chi of Eq. (S1):
 * <chi_i chi_j> = w_ij.
 *   N      number of atoms, >= 1
 *   w      pump strength, finite and >= 0
 *   alpha  exponent, finite and >= 0
 *   out    host: receives a library-owned handle; release with twa_pump_free.
 * Errors: TWA_EINVAL (N < 1, w or alpha negative or non-finite, out NULL),
 *         TWA_ENOMEM, TWA_EHIP, TWA_ENOTPSD.
 * Uses the current HIP device; blocking.
 */
TWA_API int twa_build_pump(int64_t N, double w, double alpha, twa_pump** out);

/*
 * twa_build_pump_dense -- as twa_build_pump for an arbitrary symmetric PSD
 * N x N matrix (host, row-major FP64), the generalisation the paper's
 * Perspectives note allows at unchanged cost.  w and alpha of the handle are
 * recorded as NaN.  Errors as twa_build_pump; TWA_ENOTPSD if an eigenvalue is
 * below -1e-10 * lambda_max.
 */
TWA_API int twa_build_pump_dense(int64_t N, const double* W_host, twa_pump** out);

/*
 * twa_build_model_dense -- a model handle for correlated decay: the pump W
 * and a correlated-decay matrix G (both host, row-major FP64, N x N,
 * symmetric; G must be PSD and is G_ab of SM Sec. S1 step 6), the general
 * decay matrix the paper's Perspectives name, and optionally a coherent
 * exchange Omega (host, N x N, symmetric, zero diagonal, or NULL): the
 * Hamiltonian sum_{i != j} Omega_ij sigma+_i sigma-_j of the coherent
 * dipole-dipole part of Green-tensor kernels the Perspectives mention (the
 * paper prints no equations for it; by Heisenberg's equation it adds
 * +dt (Omega s^y)_i to h^x_i and -dt (Omega s^x)_i to h^y_i in Eq. (S1)).
 * With such a handle twa_run integrates Eq. (S1) with the collective terms
 * (1/2) Gamma S^a and xi^a replaced by (1/2) sum_j G_ij s^a_j and a noise of
 * covariance G_ij (params gamma is ignored), and reports the
 * correlated-emission intensity and g2 (twa_observables I_gen, g2_gen).  The
 * decay and pump noises are drawn as one Gaussian of covariance (W + G) dt
 * (equal in law to two independent draws): the handle stores the drift
 * matrix W - G (twa_pump_copy_matrix which = 0), the PSD square root of
 * W + G (which = 1), G (which = 2) and Omega (which = 3); twa_pump_info
 * reports the eigenvalue range of W + G.  With Omega the contraction operand
 * gains a third K block (s^y, -s^x) and the corrector a second one.  Not
 * accepted by twa_adjoint; twa_run rejects it with n_lags > 0 or the split
 * precision.
 * Errors: TWA_EINVAL (bad sizes, non-finite or non-symmetric input, a nonzero
 *         diagonal of Omega), TWA_ENOTPSD (G or W + G not PSD), TWA_ENOMEM,
 *         TWA_EHIP.
 */
TWA_API int twa_build_model_dense(int64_t N, const double* W_host, const double* G_host, const double* Om_host,
                                  twa_pump** out);

/*
 * twa_build_pump_toeplitz -- a light handle of Eq. (2) for the Toeplitz fast
 * path only (twa_params pump_path = TWA_PUMP_TOEPLITZ): no dense matrices, no
 * eigendecomposition, O(1) device memory.  lam_max is the largest eigenvalue
 * of the circulant embedding (an upper bound of the largest channel rate, by
 * interlacing), lam_min is NaN.  Rejected by the dense path, twa_adjoint,
 * twa_protocol and twa_pump_copy_matrix.  Errors: TWA_EINVAL (N outside
 * 1 .. 16385, non-finite or negative w or alpha, NULL out).
 */
TWA_API int twa_build_pump_toeplitz(int64_t N, double w, double alpha, twa_pump** out);

/* Releases a handle from twa_build_pump*; NULL is ignored. */
TWA_API void twa_pump_free(twa_pump* p);

/*
 * twa_pump_info -- smallest and largest channel rate (eigenvalues of w_ij).
 * The normalised pump of the paper is w~ = lam_max / (Gamma N); the smallest
 * rate bounds the relaxation time, tau_r >= 1 / lam_min.  Any output pointer
 * may be NULL.  Errors: TWA_EINVAL for a NULL handle.
 */
TWA_API int twa_pump_info(const twa_pump* p, int64_t* N, double* lam_min, double* lam_max);

/*
 * twa_pump_copy_matrix -- copies W (which = 0), F (which = 1) or, for a model
 * handle, the decay matrix G (which = 2) or the exchange Omega (which = 3)
 * into a host row-major N x N FP64 buffer.  Errors: TWA_EINVAL, TWA_EHIP.
 */
TWA_API int twa_pump_copy_matrix(const twa_pump* p, int which, double* out_host);

/* ======================================================================
 * Trajectories: Eq. (S1) with discrete initial sampling (SM Sec. S1).
 * ====================================================================== */
typedef struct twa_params {
    const twa_pump* pump;    /* required                                          */
    double gamma;            /* collective decay rate Gamma (> 0); ignored with a  */
                             /* model handle (twa_build_model_dense)              */
    double s0z;              /* initial s^z of every spin: +1 excited, -1 ground   */
    int64_t burnin;          /* steps before the averaging window; < 0 = n_steps/2 */
    int32_t integrator;      /* TWA_INT_HEUN or TWA_INT_SIB                        */
    int32_t precision;       /* TWA_PREC_*                                         */
    int64_t n_lags;          /* two-time lags L (0 = no two-time correlation)      */
    int64_t lag_stride;      /* steps per lag; <= 0 = max(1, (n_steps-burnin)/L)   */
    int32_t point;           /* Philox point index (counter word 3, bits 8..31)    */
    int32_t tile_config;     /* < 0: automatic (heuristic; N <= 64 in FP64/FP32    */
                             /* without two-time runs the fused small-N kernel)    */
    void* stream;            /* hipStream_t, NULL = null stream                    */
    const double* init_state;/* host, optional [3][n_traj][N] (x, y, z planes):    */
                             /* replaces the discrete sampling when non-NULL       */
    int32_t timing;          /* 1: HIP events around every contraction launch      */
                             /* (fills stage*_ms); 0: only the step-loop time     */
    int32_t use_graph;       /* 1: replay the step loop from captured hipGraphs    */
    double kappa;            /* weight of the response (commutator) part in the    */
                             /* two-time correlation; default 1/4                  */
    int32_t adjoint_objectives; /* twa_adjoint: mask of 1 (<S+S->) and 2 (g2); 0 =  */
                             /* both.  The reverse sweep carries one copy per       */
                             /* objective; unselected gradients are returned NaN   */
    int32_t pump_path;       /* twa_run: TWA_PUMP_DENSE (default) or TWA_PUMP_TOEPLITZ */
    double norm_tol;         /* spin-length check: Eq. (S1) conserves |s_i|^2, so a */
                             /* run whose max_norm_dev exceeds norm_tol returns     */
                             /* TWA_EUNSTABLE (outputs written).  0 = the default  */
                             /* 1e-2; < 0 = no check (NaN/Inf are always flagged). */
                             /* The stochastic Heun integrator drifts at first     */
                             /* order in dt; the semi-implicit one keeps lengths  */
                             /* to rounding                                        */
} twa_params;

/* Fills *p with defaults: gamma 1, s0z +1, burnin -1, Heun, FP32, no lags,
 * point 0, automatic tiles, null stream, no initial state, no per-launch
 * timing, hipGraph replay on, kappa 1/4, both adjoint objectives, dense
 * pump path, norm_tol 1e-2. */
TWA_API void twa_params_default(twa_params* p);

typedef struct twa_observables {
    /* ensemble- and time-averaged TWA moments (symmetric order):
       T2 = <S+S->_TWA = <(S_x^2 + S_y^2)/4>, T3 = <S+ S^z S->_TWA,
       T4 = <S+S+S-S->_TWA, Z = <S^z>_TWA, ZZ = <S^z S^z>_TWA                */
    double T2, T3, T4, Z, ZZ;
    /* normal-ordered observables: Sz = <S^z>; SpSm = T2 + Z/2 (SM step 6);
       g2 = (T4 + 2 T3 - Z/3 + ZZ/2 - 4 T2/3) / SpSm^2 (Eq. (S2), main text) */
    double Sz, SpSm, g2;
    /* delete-one-block jackknife standard errors (32 contiguous blocks of
       trajectories, fewer if n_traj < 32), same order as above              */
    double T2_se, T3_se, T4_se, Z_se, ZZ_se, Sz_se, SpSm_se, g2_se;
    int64_t n_samples;       /* window samples per trajectory                       */
    int64_t n_lags;          /* lags written                                       */
    int64_t lag_stride;      /* steps per lag                                      */
    double max_norm_dev;     /* max over spins of | |s|^2(end) - |s|^2(start) |    */
    double step_criterion;   /* max(Gamma N, lam_max) dt; the paper asks < 0.05    */
    int32_t nan_flag;        /* 1 if a NaN/Inf was seen                            */
    int32_t tile_config;     /* tile configuration used (TWA_TILE_FUSED: the fused */
                             /* small-N kernel, every step in one launch)          */
    double kernel_ms;        /* device time of the step loop (HIP events)          */
    double stage1_ms;        /* timing = 1: summed device time of the predictor    */
    int64_t stage1_launches; /* contraction launches (HIP events around each) and  */
    double stage2_ms;        /* of the corrector contraction launches              */
    int64_t stage2_launches;
    double gemm_flops;       /* algorithmic flops of all contractions of the run   */
    /* two-time (n_lags > 0): C(l) = Csym(l) + kappa i (chi_xx + chi_yy
       + i chi_yx - i chi_xy) (Eq. (S3) and the Kubo correction after it);
       spectrum S(omega) = 2 Re int_0^inf e^{i omega t} C(t) dt (trapezoid on
       the lag grid, zero padded to 8 L); linewidth = its FWHM (main text)   */
    double linewidth;        /* FWHM of the spectrum of C                          */
    double linewidth_sym;    /* FWHM of the spectrum of Csym alone                 */
    double adjoint_fwd_ms;   /* twa_adjoint: device time of the checkpointed       */
    double adjoint_bwd_ms;   /* forward run and of the reverse sweep (recompute    */
                             /* included); kernel_ms is their sum                  */
    /* correlated decay (model handles; NaN otherwise), SM Sec. S1 step 6:
       I_gen = <sum_ab G_ab s+_a s-_b> = <E2>_TWA + (1/2) sum_a G_aa <s^z_a>_TWA;
       g2_gen = sum_abcd G_ad G_bc <s+_a s+_b s-_c s-_d> / I_gen^2 from the
       printed four-point expression; jackknife errors as above              */
    double I_gen, g2_gen, I_gen_se, g2_gen_se;
} twa_observables;

/* Optional host output buffers of twa_run (any may be NULL). */
typedef struct twa_outputs {
    double* corr_blocks;     /* [L][J][2] block sums of the symmetric part
                                (1/4)(S_x + i S_y)(t0 + l m dt) (S_x - i S_y)(t0) */
    double* chi_blocks;      /* [L][J][4] block sums of sum_i ds^a_i of the
                                response copies: xx, yx, xy, yy                   */
    double* traj_moments;    /* [n_traj][5] per-trajectory window averages of
                                T2, T3, T4, Z, ZZ                                 */
    double* final_state;     /* [3][n_traj][N] x, y, z planes at the last step    */
    int32_t* n_blocks;       /* receives J                                        */
    double* traj_gen;        /* model handles: [n_traj][9] window averages of E2,
                                E2^2, E2 D, Q3, R, D^2, U, V, D with
                                E2 = sum_ab G_ab s+_a s-_b, D = sum_a G_aa s^z_a,
                                Q3 = sum_b s^z_b |(G s+)_b|^2, R = sum_a G_aa^2 s^z_a,
                                U = s^z . (G o G) s^z, V = Re sum_ab G_aa G_ab s+_a s-_b */
} twa_outputs;

/*
 * twa_run -- integrate n_traj independent trajectories of Eq. (S1) for
 * n_steps steps of size dt and accumulate the observables.
 *   Noise: Philox4x32-10 with key (seed low word, seed high word) and
 *   counter (c0, c1, c2, c3), c3 = tag | (point << 8); Box-Muller turns each
 *   pair of words into a pair of normals.  Step n (0-based), trajectory k:
 *   zeta^x, zeta^y of spin 2m from words (0, 1) and of spin 2m+1 from words
 *   (2, 3) of counter (m, k, n, tag 0); g^x, g^y from words (0, 1) of
 *   (0, k, n, tag 1).  xi^a dt -> sqrt(Gamma dt) g^a (one collective normal
 *   pair per trajectory and step), chi^a dt -> sqrt(dt) F zeta^a (N normal
 *   pairs per trajectory and step).  Initial signs of s^x_i, s^y_i: bits
 *   2j, 2j+1 (j = i mod 64) of counter (i / 64, k, 0, tag 2).
 *   Integrator: stochastic Heun (Euler predictor, trapezoidal corrector with
 *   the same noise increments).
 *   Window: states after steps burnin+1 .. n_steps are averaged.
 *   Two-time (n_lags > 0): origin at the state after `burnin` steps; two
 *   tangent-linear response copies seeded with ds = x^ and ds = y^ on every
 *   spin (the eps -> 0 limit of the SM's shifted copies) run alongside;
 *   lag l samples the state after burnin + l * stride steps.
 *   out   host, required: scalar results.
 *   outs  host, optional: per-block / per-trajectory arrays.
 *   Model handle (twa_build_model_dense): correlated decay in place of the
 *   collective terms; every observed state also passes through G [s^x, s^y]
 *   and (G o G) s^z contractions in the run's contraction precision, and the
 *   correlated-emission intensity and g2 are reported (I_gen, g2_gen).
 * Errors: TWA_EINVAL (NULL pump/out, n_traj < 1, n_steps < 0, dt <= 0,
 *         burnin > n_steps, gamma <= 0 without a model handle, unknown
 *         precision, lags that do not fit: (n_lags - 1) * stride >
 *         n_steps - burnin, n_lags > 0 with a model handle), TWA_ENOMEM,
 *         TWA_EHIP, TWA_EUNSTABLE.
 * Deterministic: identical inputs give bitwise identical outputs.
 */
TWA_API int twa_run(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps,
                    uint64_t seed, twa_observables* out, const twa_outputs* outs);

/*
 * twa_run_noalloc -- twa_run for callers that cannot allocate device memory:
 * tight serving loops, harnesses that forbid hipMalloc, processes whose
 * device memory another allocator owns.  It calls no allocating routine
 * (hipMalloc, hipFree or a library routine that allocates); it does end
 * with a copy of the scalar results to the host and a synchronisation of
 * the caller's stream, so it cannot itself be recorded under hipGraph
 * stream capture (call it outside a capture).  Every buffer of the run
 * is carved from a file-scope device array of TWA_NOALLOC_SCRATCH_BYTES that
 * each device holds until the process ends (its address taken once per
 * device), and the jackknife block sums are formed on the device.  Same
 * kernels and results as twa_run (bit for bit) for: a pump from
 * twa_build_pump or twa_build_pump_dense, Heun or the semi-implicit scheme,
 * any precision, n_lags = 0, no init_state; no hipGraph replay and no timing
 * (kernel_ms is NaN).  The caller passes the stream (NULL = null stream).
 * Calls share the device's array; within one process the library's lock
 * keeps them from overlapping (calls from several processes would race).
 * Errors: TWA_EINVAL (as twa_run, and for the unsupported options above),
 *         TWA_ENOMEM (the run's buffers exceed the scratch size; the message
 *         states the bytes needed), TWA_EHIP, TWA_EUNSTABLE.
 */
#define TWA_NOALLOC_SCRATCH_BYTES (64u << 20)
TWA_API int twa_run_noalloc(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                            twa_observables* out);

/* ======================================================================
 * Batched phase-diagram scan: many independent (N, w, alpha) points.
 * ====================================================================== */
typedef struct twa_point {
    int64_t N;
    double w, alpha;
    double dt;
    uint64_t seed;
} twa_point;

typedef struct twa_batch_opts {
    int64_t n_traj;          /* trajectories per point                           */
    int64_t n_steps;         /* steps per point                                  */
    int64_t burnin;          /* < 0: n_steps / 2                                  */
    double gamma;
    double s0z;
    int32_t precision;       /* TWA_PREC_FP64 / FP32 / BF16 / FP16 / BF16X3     */
    int32_t use_graph;       /* capture the step loop in hipGraphs (default 1)   */
    int32_t steps_per_graph; /* steps captured per graph replay (<= 0: 16)       */
    const char* tune_cache;  /* autotuner cache file (NULL: no cache)            */
    void* stream;            /* hipStream_t                                      */
    int32_t integrator;      /* TWA_INT_HEUN (default) or TWA_INT_SIB            */
    double norm_tol;         /* as twa_params.norm_tol, per point (0: 1e-2)      */
    int64_t n_lags;          /* two-time lags per point, as twa_params (0: none; */
                             /* Heun only)                                       */
    int64_t lag_stride;      /* as twa_params                                    */
    double kappa;            /* as twa_params (default 1/4)                      */
    int32_t tile_config;     /* < 0: autotuned per N bucket; >= 0: one tile      */
                             /* configuration (0..3, or 7 without FP64) for all  */
    int64_t progress_every;  /* > 0: print a progress line to stderr every this  */
                             /* many steps (the host then waits for the device   */
                             /* at those steps); 0: silent                       */
    const twa_outputs* outputs; /* host, optional: array of n_points twa_outputs */
                             /* (traj_moments, final_state, corr_blocks,         */
                             /* chi_blocks, n_blocks; traj_gen is not used)      */
} twa_batch_opts;

/* Defaults: 512 trajectories, 1000 steps, burn-in n_steps/2, gamma 1, s0z +1,
 * FP32, graphs of 16 steps, no cache, own stream, Heun, norm_tol 1e-2, no
 * lags, kappa 1/4, autotuned tiles, silent, no per-point arrays. */
TWA_API void twa_batch_opts_default(twa_batch_opts* o);

/*
 * twa_run_batch -- an uneven phase-diagram scan (main text, results: the
 * (w~, alpha) diagrams and the N dependence): every point of `pts` is a full
 * ensemble of Eq. (S1) trajectories with its own pump of Eq. (2) (built
 * internally), its own step size and seed, and Philox point index = its
 * position in `pts`; all points share n_traj, n_steps, the window and the
 * lags.  The points are split into N buckets (N <= 128, N <= 1024, larger);
 * every bucket advances in grouped persistent launches (one per stage and
 * step, over the LPT-ordered tiles of all its points) with the tile
 * configuration the autotuner measured fastest for it (cached on disk when a
 * cache file is given), each bucket on its own stream branch of one captured
 * hipGraph per steps_per_graph steps.  With n_lags > 0 every point also
 * carries the two response copies of its two-time correlation and reports its
 * linewidth.  Results equal those of twa_run on each point with the same tile
 * configuration, bit for bit.  outs[i] receives point i's observables.
 * Errors as twa_run; TWA_EUNSTABLE if any point is unstable (all outputs
 * written).
 */
TWA_API int twa_run_batch(const twa_point* pts, int n_points, const twa_batch_opts* o,
                          twa_observables* outs);

/* ======================================================================
 * Adjoint: pathwise gradients at fixed noise.
 * ====================================================================== */
/*
 * twa_adjoint -- forward run of twa_run (no two-time) with the state
 * checkpointed every `ckpt_every` steps, then a reverse sweep through the
 * Heun steps (each segment recomputed from its checkpoint) giving the
 * pathwise derivatives, at the fixed Philox stream, of the steady-state
 * <S+S-> (SpSm) and g2 with respect to w and alpha of an Eq. (2) pump:
 *   grads[0] = dSpSm/dw, grads[1] = dSpSm/dalpha,
 *   grads[2] = dg2/dw,   grads[3] = dg2/dalpha.
 * The observables of the forward run are written to *out.  Requires a pump
 * from twa_build_pump with w > 0 and the Heun integrator; precision FP64,
 * FP32 or split BF16 (TWA_PREC_BF16X3: every contraction, forward and
 * reverse, with its operands in the hi, lo, hi form).  Errors as twa_run.
 */
TWA_API int twa_adjoint(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps,
                        uint64_t seed, int32_t ckpt_every, twa_observables* out,
                        double* grads);

/*
 * twa_tangent_w -- forward-mode counterpart of twa_adjoint for the pump
 * amplitude w alone: the pathwise derivatives, at the fixed Philox stream,
 *   grads[0] = dSpSm/dw, grads[1] = dg2/dw, grads[2] = dSz/dw
 * of the steady-state observables of twa_run (written to *out), from one
 * tangent-linear copy ds/dw propagated beside the Heun steps of Eq. (S1) with
 * the field's own derivative dH/dw = Y/w - Q/(2w) as its source (W is linear
 * and its PSD square root F square-root homogeneous in w at fixed alpha; Y
 * the contraction output of a stage, Q its noise part).  About 5/3 of a
 * forward run in contraction work, no checkpoint store; the cheaper choice
 * for one parameter (the threshold search in w).  Requires a pump from
 * twa_build_pump with w > 0; Heun, no lags, any precision (split BF16
 * included: the tangent's operands in the hi, lo, hi form).  grads: host,
 * 3 doubles.  Errors as twa_adjoint.
 */
TWA_API int twa_tangent_w(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                          twa_observables* out, double* grads);

/* ======================================================================
 * The paper's protocol and threshold quantities.
 * ====================================================================== */
/* Objectives of the threshold search (main text, results): the coherent-light
 * cutoff g2 = 1.08 at fixed N and the superradiant intensity <S+S-> = N. */
#define TWA_OBJ_G2       0   /* g2 of the steady state                            */
#define TWA_OBJ_SPSM_N   1   /* <S+S-> / N of the steady state                    */

typedef struct {
    double dt;               /* cfl / max(Gamma N, lambda_max): the step criterion of
                                the main text's methods paragraph (< 0.05)          */
    double tau_s;            /* preparation time: 10/Gamma for alpha < 1, 10/lambda_min
                                for alpha >= 1 (main text); with finite_size,
                                10 / [w (2 eta(alpha) - 1)] (SM Sec. S1)            */
    double tau;              /* averaging window 5/Gamma                           */
    int64_t n_prep;          /* ceil(tau_s / dt - 1e-9): burn-in steps              */
    int64_t n_window;        /* ceil(tau / dt - 1e-9): window steps                 */
    double wt;               /* normalised pump lambda_max / (Gamma N)              */
    double lam_min, lam_max; /* channel rates of the pump                          */
} twa_protocol_t;

/*
 * twa_protocol -- the protocol of one point of the paper's scans for a pump
 * from twa_build_pump (finite_size also needs its w and alpha; eta is the
 * Dirichlet eta function, computed by Borwein's alternating-series method).
 * cfl must be in (0, 0.05).  Errors: TWA_EINVAL (null pointers, gamma <= 0,
 * cfl outside (0, 0.05), finite_size with 2 eta(alpha) - 1 <= 0 or a dense
 * pump).
 */
TWA_API int twa_protocol(const twa_pump* pump, double gamma, double cfl, int32_t finite_size,
                         twa_protocol_t* out);

typedef struct {
    int32_t objective;       /* TWA_OBJ_G2 or TWA_OBJ_SPSM_N                       */
    double target;           /* e.g. 1.08 for g2, 1.0 for <S+S->/N                 */
    double w_lo, w_hi;       /* bracket of the pump amplitude w of Eq. (2),
                                0 < w_lo < w_hi, objective - target changing sign  */
    double tol_w;            /* stop once the Newton correction is below tol_w      */
    int32_t max_iter;        /* derivative evaluations at most                      */
    int32_t ckpt_every;      /* checkpoint interval of twa_adjoint                  */
    int32_t derivative;      /* TWA_DERIV_FORWARD (default): twa_tangent_w;         */
                             /* TWA_DERIV_ADJOINT: the reverse sweep of twa_adjoint */
} twa_threshold_opts;

#define TWA_DERIV_FORWARD 0
#define TWA_DERIV_ADJOINT 1

TWA_API void twa_threshold_opts_default(twa_threshold_opts* o);

/*
 * twa_find_threshold -- the pump amplitude w at which the fixed-noise
 * steady-state objective of twa_run (same seed for every w, so the
 * objective is a smooth function of w) equals o->target, by Newton steps
 * with the pathwise derivative (twa_tangent_w, or twa_adjoint with
 * o->derivative = TWA_DERIV_ADJOINT), kept inside a bracket that
 * is bisected whenever a Newton step leaves it.  The pump is factorised once
 * (at w_hi); other amplitudes scale it exactly (W ~ w, F ~ sqrt(w)).  p gives
 * gamma, s0z, burnin, precision, point and tile_config; p->pump is ignored.
 * Outputs: *w_root, *f_root = objective(w_root) - target, *n_iter = gradient
 * evaluations used (any output pointer may be NULL).  Errors as twa_adjoint;
 * TWA_ENOROOT if the bracket has no sign change or max_iter is reached.
 */
TWA_API int twa_find_threshold(int64_t N, double alpha, const twa_params* p, int64_t n_traj, double dt,
                               int64_t n_steps, uint64_t seed, const twa_threshold_opts* o, double* w_root,
                               double* f_root, int32_t* n_iter);

/*
 * twa_g2_min -- the g2_min protocol of the paper (main text, results): g2 at
 * n_points equally spaced normalised pumps w~ in [wt_lo, wt_hi], every point
 * run with its own twa_protocol (n_prep burn-in steps + n_window averaged
 * steps, same seed), and the smallest of them.  wt_out[n_points] and
 * g2_out[n_points] (host, may be NULL) receive the curve.  p as in
 * twa_find_threshold.  Errors as twa_run and twa_protocol.
 */
TWA_API int twa_g2_min(int64_t N, double alpha, const twa_params* p, int64_t n_traj, uint64_t seed,
                       int32_t n_points, double wt_lo, double wt_hi, double cfl, int32_t finite_size,
                       double* wt_out, double* g2_out, double* wt_min, double* g2_min);

/* ======================================================================
 * Kernel-level entry points used by the parity tests.
 * ====================================================================== */
/*
 * twa_philox -- raw Philox4x32-10 blocks on the device: for j < n,
 * out[4j .. 4j+3] = Philox4x32-10(ctr[4j .. 4j+3], key = (key0, key1)).
 * ctr, out: device, uint32, 4n each.  Errors: TWA_EINVAL, TWA_EHIP.
 */
TWA_API int twa_philox(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1,
                       uint32_t* out, void* stream);

/*
 * twa_noise -- the Gaussians the step kernels draw for one step: zeta^x,
 * zeta^y of every (trajectory, spin) and g^x, g^y of every trajectory, in
 * FP64 (fp64 = 1) or FP32 Box-Muller, written as doubles.
 *   zeta: device [2][n_traj][N]; g: device [2][n_traj].  Errors as above.
 */
TWA_API int twa_noise(uint64_t seed, int64_t step, int32_t point, int64_t n_traj, int64_t N,
                      int32_t fp64, double* zeta, double* g, void* stream);

/* Last error message of the calling thread ("" if none). */
TWA_API const char* twa_last_error(void);

/* Library version string. */
TWA_API const char* twa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TWA_H */
