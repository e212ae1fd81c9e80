"""FP64 CPU oracle for the dissipative Truncated-Wigner (TWA) trajectory method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library (``paper_2608_10075_amd``) and imports nothing from it.

What it computes, each step following the paper (Chelpanova, Stefanini,
O'Keeffe, Marino, "Phase diagram of lasing under correlated pump from
GPU-accelerated Truncated Wigner dynamics"):

* ``pump``        -- the pump-rate matrix of Eq. (2), its channel decomposition
                     (main text, paragraph after Eq. (2)) and the symmetric PSD
                     square root used to colour the pump noise of Eq. (S1);
                     eigenvalue laws of Eq. (3) and the Dirichlet-eta estimate
                     of the smallest channel rate.
* ``philox``      -- the counter-based random numbers (Philox4x32-10, Salmon et
                     al., SC'11) and Box-Muller Gaussians that drive the noises
                     of Eq. (S1); the paper names no generator, the counter
                     layout is this project's reading.
* ``twa``         -- discrete initial sampling (SM Sec. S1, step 3), the
                     stochastic equations of motion Eq. (S1) integrated with the
                     Stratonovich stochastic Heun scheme, time-averaged
                     observables (SM Sec. S1 steps 5-6 and the closing remark on
                     time averaging), and the two-time correlation with the
                     three-copy response construction (SM Sec. S1, Eq. (S3) and
                     following).
* ``observables`` -- the normal-ordering conversions (SM Sec. S1 step 6,
                     Eq. (S2)), g2 (main text, Observables and method), the
                     jackknife error bars and the spectrum / linewidth.
* ``grad``        -- pathwise (fixed-noise) derivatives of the steady-state
                     observables with respect to w and alpha by forward-mode
                     tangent propagation, and the Sylvester solve for dF/dalpha.
* ``lindblad``    -- brute-force density-matrix Lindbladian of Eq. (1) for tiny
                     N (optionally with a correlated-decay matrix in place of
                     the collective term), used only to pin the oracle's
                     equations of motion.
* ``decay``       -- correlated decay (the general-matrix extension named in
                     the Perspectives): the step's matrices W - G and
                     sqrt(W + G), and the intensity and four-point function of
                     correlated emission (SM Sec. S1 step 6) with jackknife.
* ``toeplitz``    -- not in the paper: Eq. (2) applied through its circulant
                     embedding (FFT products) with the pump noise drawn from the
                     embedding (equal in law to the dense path's).
* ``protocol``    -- the paper's time-step criterion, preparation time and
                     window, and the threshold / g2-minimum searches.
* ``closed_forms``-- the alpha=0 closed forms (noiseless superradiant decay and
                     the stationary law of the collective spin) used as pins.

Parity status: every public function is pinned by a ``-m "not gpu"`` test
under ``tests/`` against a value that does not come from this package (a
published test vector, a closed form, a brute-force computation, an exact
enumeration or a textbook solver).  No function here is "parity unpinned".
"""
