// twa_adjoint: pathwise gradients of the steady-state <S+S-> and g2 with
// respect to w and alpha of the pump of Eq. (2), at fixed Philox noise, by a
// reverse sweep through the stochastic Heun steps of Eq. (S1).
//
// Forward: an ordinary run that also stores the state every `ckpt_every`
// steps.  Backward, segment by segment from the last: the segment's steps are
// recomputed from its checkpoint, storing per step the state s, the predictor
// increment D, the contraction outputs Y1 = A [s; zeta], Y2 = Y1 + A_left D,
// the noise part Q = -sqrt(dt) F zeta and the alpha-derivatives of Y1 and Y2
// (A_alpha = [-dt/2 dW/dalpha | -sqrt(dt) dF/dalpha]); then the cotangent of
// the state is carried back through each step:
//   corrector (kind ADJ2):  mu2 = lam'/2, nu2 = df/dH^T mu2 at s~,
//       lam~ = df/ds^T mu2 + (Gamma dt/2) sum(nu2) + A_left nu2,
//       mu1 = mu2 + lam~, R = lam' + lam~, nu1 = df/dH^T mu1 at s
//   predictor (kind ADJ1):  lam = R + df/ds^T mu1 + (Gamma dt/2) sum(nu1) + A_left nu1 + source,
// with the source the derivative of the time- and ensemble-averaged moments
// of the observed state.  The parameters enter only through the fields H,
// dH/dw = Y/w - Q/(2w) (W is linear and F is sqrt-homogeneous in w) and
// dH/dalpha = A_alpha [s; zeta], so dJ/dtheta = sum over steps of
// <nu1, dH1/dtheta> + <nu2, dH2/dtheta>, accumulated per tile in FP64.
// Both objectives (<S+S-> and g2, whose source follows the quotient rule on
// the forward ensemble moments) are carried together as two copies.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "twa_device.h"
#include "twa_internal.h"
#include "twa_run.h"

namespace twa {

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// dW/dalpha = -log(1 + |i-j|) w_ij (derivative of Eq. (2)), column-major = row-major
__global__ void dw_dalpha_kernel(const double* W, int64_t N, double* Wa) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t i = t / N, j = t % N;
    Wa[t] = -log1p((double)(i > j ? i - j : j - i)) * W[t];
}

// X'_ij = T_ij / (r_i + r_j), zero where the denominator vanishes (column-major T)
__global__ void sylvester_scale_kernel(double* T, const double* r, int64_t N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t col = t / N, row = t % N;
    const double d = r[row] + r[col];
    T[t] = d > 0 ? T[t] / d : 0.0;
}

__global__ void symmetrize_kernel2(int64_t N, double* F) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t i = t / N, j = t % N;
    if (j <= i) return;
    const double v = 0.5 * (F[i * N + j] + F[j * N + i]);
    F[i * N + j] = v;
    F[j * N + i] = v;
}

__global__ void set_step_kernel(int64_t* step, int64_t v) { step[0] = v; }

// write the s-part of the operand from a state (split form: hi, lo, hi
// blocks of P each)
template <int PREC>
__global__ void state_to_op_kernel(const typename Prec<PREC>::S* s, int64_t P, int64_t Bp,
                                   typename Prec<PREC>::G* Xop) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bp * P) return;
    const int64_t k = t / P, i = t % P, SP = Bp * P, ld = 2 * P * Prec<PREC>::SPLIT;
    put_op<PREC>(Xop + opcol(k, 0) * ld + i, P, s[t]);
    put_op<PREC>(Xop + opcol(k, 1) * ld + i, P, s[SP + t]);
}

// nu2 = df/dH^T (lam/2) at the predictor state s~ = s + D, as the operand of
// the corrector's adjoint contraction, with its spin sums per M tile.
// grid (ceil(Bp/4), nmt, 2 copies), 256 threads = 4 trajectories x 64 lanes
template <int PREC>
__global__ __launch_bounds__(256) void prep_nu2_kernel(const typename Prec<PREC>::S* lam,
                                                       const typename Prec<PREC>::S* s,
                                                       const typename Prec<PREC>::S* d, int64_t P, int64_t Bp,
                                                       int64_t nmt, int64_t mtile, int64_t C2,
                                                       typename Prec<PREC>::G* op, typename Prec<PREC>::S* part) {
    typedef typename Prec<PREC>::S S;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * 4 + wv;
    const int64_t mt = blockIdx.y;
    const int cp = blockIdx.z;
    if (k >= Bp) return;   // uniform per wave
    const int64_t SP = Bp * P;
    const S* l = lam + (int64_t)cp * 3 * SP;
    const int64_t ld = P * Prec<PREC>::SPLIT;   // operand column pitch (split: hi, lo, hi blocks)
    typename Prec<PREC>::G* o = op + (int64_t)cp * C2 * ld;
    S sx = 0, sy = 0;
    for (int64_t i = mt * mtile + lane; i < (mt + 1) * mtile; i += 64) {
        const int64_t e = k * P + i;
        const S px = s[e] + d[e], py = s[SP + e] + d[SP + e], pz = s[2 * SP + e] + d[2 * SP + e];
        const S ux = S(0.5) * l[e], uy = S(0.5) * l[SP + e], uz = S(0.5) * l[2 * SP + e];
        const S nx = ux * pz - uz * px, ny = uy * pz - uz * py;
        put_op<PREC>(o + opcol(k, 0) * ld + i, P, nx);
        put_op<PREC>(o + opcol(k, 1) * ld + i, P, ny);
        sx += nx;
        sy += ny;
    }
    for (int w = 32; w > 0; w >>= 1) {
        sx += __shfl_xor(sx, w);
        sy += __shfl_xor(sy, w);
    }
    if (lane == 0) {
        S* pp = part + (int64_t)cp * 3 * nmt * Bp;
        pp[(0 * nmt + mt) * Bp + k] = sx;
        pp[(1 * nmt + mt) * Bp + k] = sy;
        pp[(2 * nmt + mt) * Bp + k] = S(0);
    }
}

// cotangent of the last state: the observation source alone
template <typename S>
__global__ void src_init_kernel(const S* part, int64_t N, int64_t B, int64_t P, int64_t Bp, int64_t nmt, S c00,
                                S c01, S c02, S c03, S c04, S c10, S c11, S c12, S c13, S c14, S scale, int on,
                                int64_t ncopy, S* lam) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncopy * Bp * P) return;
    const int cp = (int)(t / (Bp * P));
    const int64_t r = t % (Bp * P), k = r / P, i = r % P, SP = Bp * P;
    S ox = 0, oy = 0, oz = 0;
    if (on && k < B && i < N) {
        S sx = 0, sy = 0, sz = 0;
        for (int64_t q = 0; q < nmt; ++q) {
            sx += part[(0 * nmt + q) * Bp + k];
            sy += part[(1 * nmt + q) * Bp + k];
            sz += part[(2 * nmt + q) * Bp + k];
        }
        const S cf[5] = {cp ? c10 : c00, cp ? c11 : c01, cp ? c12 : c02, cp ? c13 : c03, cp ? c14 : c04};
        const S T2 = S(0.25) * (sx * sx + sy * sy);
        const S gt = S(0.5) * cf[0] + S(0.5) * cf[1] * sz + cf[2] * T2;
        ox = scale * gt * sx;
        oy = scale * gt * sy;
        oz = scale * (cf[1] * T2 + cf[3] + S(2) * cf[4] * sz);
    }
    S* l = lam + (int64_t)cp * 3 * SP;
    l[r] = ox;
    l[SP + r] = oy;
    l[2 * SP + r] = oz;
}

template <int PREC>
int state_to_op(const Geometry& g, const void* s, void* Xop, hipStream_t st) {
    hipLaunchKernelGGL(state_to_op_kernel<PREC>, dim3(nblk(g.Bp * g.P, 256)), dim3(256), 0, st,
                       static_cast<const typename Prec<PREC>::S*>(s), g.P, g.Bp,
                       static_cast<typename Prec<PREC>::G*>(Xop));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <int PREC>
int prep_nu2(const Geometry& g, const void* lam, const void* s, const void* d, void* op, void* part, int ncopy,
             hipStream_t st) {
    typedef typename Prec<PREC>::S S;
    dim3 grid(nblk(g.Bp, 4), (unsigned)g.nmt, (unsigned)ncopy);
    hipLaunchKernelGGL(prep_nu2_kernel<PREC>, grid, dim3(256), 0, st, static_cast<const S*>(lam),
                       static_cast<const S*>(s), static_cast<const S*>(d), g.P, g.Bp, g.nmt, g.P / g.nmt, g.C2,
                       static_cast<typename Prec<PREC>::G*>(op), static_cast<S*>(part));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <int PREC>
int src_init(const Geometry& g, const void* part, const double (*cf)[5], double scale, int on, void* lam,
             int ncopy, hipStream_t st) {
    typedef typename Prec<PREC>::S S;
    hipLaunchKernelGGL(src_init_kernel<S>, dim3(nblk((int64_t)ncopy * g.Bp * g.P, 256)), dim3(256), 0, st,
                       static_cast<const S*>(part), g.N, g.B, g.P, g.Bp, g.nmt, (S)cf[0][0], (S)cf[0][1],
                       (S)cf[0][2], (S)cf[0][3], (S)cf[0][4], (S)cf[1][0], (S)cf[1][1], (S)cf[1][2], (S)cf[1][3],
                       (S)cf[1][4], (S)scale, on, (int64_t)ncopy, static_cast<S*>(lam));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

// dF/dalpha from F X + X F = dW/dalpha, solved in the eigenbasis of W:
// X = V [(V^T dW V)_ij / (r_i + r_j)] V^T, r = sqrt(lambda+) (FP64, one-time)
int dfactor_dalpha(const twa_pump* p, double* Wa, double* Fa, hipStream_t st) {
    const int64_t N = p->N;
    const size_t bytes = (size_t)N * N * sizeof(double);
    double *T = nullptr, *U = nullptr, *r = nullptr;
    rocblas_handle h = nullptr;
    int rc = TWA_OK;
    std::vector<double> rr((size_t)N);
    const double tol = 8.0 * (double)N * DBL_EPSILON * std::max(p->lam_max, 0.0);
    for (int64_t j = 0; j < N; ++j) rr[(size_t)j] = p->lam[j] > tol ? std::sqrt(p->lam[j]) : 0.0;
    const double one = 1.0, zero = 0.0;
    const rocblas_int n = (rocblas_int)N;
    if (hipMalloc(&T, bytes) != hipSuccess || hipMalloc(&U, bytes) != hipSuccess ||
        hipMalloc(&r, N * sizeof(double)) != hipSuccess) {
        set_error("twa_adjoint: device allocation for dF/dalpha failed");
        rc = TWA_ENOMEM;
        goto done;
    }
    if (rocblas_create_handle(&h) != rocblas_status_success || rocblas_set_stream(h, st) != rocblas_status_success) {
        set_error("twa_adjoint: rocblas_create_handle failed");
        rc = TWA_EHIP;
        goto done;
    }
    hipLaunchKernelGGL(dw_dalpha_kernel, dim3(nblk(N * N, 256)), dim3(256), 0, st, p->W, N, Wa);
    if (hipMemcpyAsync(r, rr.data(), N * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess ||
        rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &one, p->V, n, Wa, n, &zero, U,
                      n) != rocblas_status_success ||
        rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, U, n, p->V, n, &zero, T, n) !=
            rocblas_status_success) {
        set_error("twa_adjoint: rocBLAS failed in dF/dalpha");
        rc = TWA_EHIP;
        goto done;
    }
    hipLaunchKernelGGL(sylvester_scale_kernel, dim3(nblk(N * N, 256)), dim3(256), 0, st, T, r, N);
    if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, p->V, n, T, n, &zero, U, n) !=
            rocblas_status_success ||
        rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, U, n, p->V, n, &zero, Fa,
                      n) != rocblas_status_success) {
        set_error("twa_adjoint: rocBLAS failed in dF/dalpha");
        rc = TWA_EHIP;
        goto done;
    }
    hipLaunchKernelGGL(symmetrize_kernel2, dim3(nblk(N * N, 256)), dim3(256), 0, st, N, Fa);
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("twa_adjoint: dF/dalpha kernels failed");
        rc = TWA_EHIP;
    }
done:
    if (h) rocblas_destroy_handle(h);
    hipFree(T);
    hipFree(U);
    hipFree(r);
    return rc;
}

struct SegStore {
    // per step slot j of a segment (planes of Bp * P state elements)
    void* s = nullptr;      // [K+1][3]
    void* d = nullptr;      // [K][3]
    void* y1 = nullptr;     // [K][2]
    void* y2 = nullptr;     // [K][2]
    void* q = nullptr;      // [K][2]
    void* ya1 = nullptr;    // [K][2]
    void* ya2 = nullptr;    // [K][2]
    void* partS = nullptr;  // [K+1][3][nmt][Bp]
    void* partP = nullptr;  // [K][3][nmt][Bp]
    void* g = nullptr;      // [K][2][Bp]
    void* ckpt = nullptr;   // [nseg][3] planes
    void* ckpt_part = nullptr;  // [nseg][3][nmt][Bp] spin sums of the checkpointed states
    void* Aa = nullptr;     // G [P][2P]
    void* lam = nullptr;    // [2][3] planes
    void* M1 = nullptr;
    void* Rb = nullptr;
    void* nu2 = nullptr;    // G [2][C2][P]
    void* nu1 = nullptr;
    void* nu2p = nullptr;   // [2][3][nmt][Bp]
    void* nu1p = nullptr;
    double* gacc = nullptr; // [2][2][nmt][Bp]
    void release() {
        void* ptrs[] = {s,    d,  y1,  y2, q,   ya1, ya2,  partS, partP, g,   ckpt,
                        ckpt_part, Aa, lam, M1, Rb, nu2, nu1, nu2p, nu1p, gacc};
        for (void* p : ptrs) hipFree(p);
    }
};

int dalloc0(void** p, size_t bytes, hipStream_t st) {
    if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) {
        *p = nullptr;
        set_error("twa_adjoint: device allocation of " + std::to_string(bytes) + " bytes failed");
        return TWA_ENOMEM;
    }
    if (hipMemsetAsync(*p, 0, bytes ? bytes : 16, st) != hipSuccess) {
        set_error("twa_adjoint: hipMemsetAsync failed");
        return TWA_EHIP;
    }
    return TWA_OK;
}

template <int PREC>
int adjoint_impl(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed, int K,
                 twa_observables* out, double* grads) {
    typedef typename Prec<PREC>::S S;
    const twa_pump* pump = p->pump;
    const int64_t N = pump->N, B = n_traj;
    const int64_t burnin = p->burnin < 0 ? n_steps / 2 : p->burnin;
    const int cfg = p->tile_config >= 0 ? p->tile_config : pick_tile_cfg(p->precision, N, B);
    const Geometry g = make_geometry(p->precision, cfg, N, B);
    const int J = (int)std::min<int64_t>(32, B);
    const int64_t nseg = (n_steps + K - 1) / K;
    // objectives carried by the reverse sweep (0 = <S+S->, 1 = g2), one copy each
    const int mask = p->adjoint_objectives == 0 ? 3 : p->adjoint_objectives;
    int obj[2] = {0, 1}, nobj = 0;
    if (mask & 1) obj[nobj++] = 0;
    if (mask & 2) obj[nobj++] = 1;
    const size_t se = sizeof(S), ge = (size_t)gemm_elt_bytes(p->precision);
    // K extent of one operand block: P, or 3P in the split form (hi, lo, hi)
    const int64_t KP = g.P * Prec<PREC>::SPLIT;
    const size_t plane = (size_t)g.Bp * g.P * se;
    const size_t partsz = (size_t)3 * g.nmt * g.Bp * se;

    hipStream_t st = (hipStream_t)p->stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) {
            set_error("twa_adjoint: hipStreamCreate failed (no usable GPU?)");
            return TWA_EHIP;
        }
        st = own;
    }
    EnsembleBuffers b;
    SegStore m;
    double *Wa = nullptr, *Fa = nullptr;
    int rc = TWA_OK;
    int cur = 0;
    StepConsts c;
    double cf[2][5];
    double scale = 0;
    std::vector<double> hmom, hg;
    std::vector<float> hdiag;
    const int nblk_fin = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (B * N + 255) / 256));
    double fwd_norm_dev = 0;
    bool fwd_nan = false;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    float fwd_ms = 0.f, bwd_ms = 0.f;
    c.c1 = 0.5 * p->gamma * dt;
    c.c2 = std::sqrt(p->gamma * dt);
    c.s0z = p->s0z;
    c.key0 = (uint32_t)(seed & 0xffffffffu);
    c.key1 = (uint32_t)(seed >> 32);
    c.point = p->point;
    c.burnin = burnin;
    c.lag_stride = 1;
    c.n_lags = 0;
    c.J = J;

#define TWA_TRY(expr)                              \
    do {                                           \
        if ((rc = (expr)) != TWA_OK) goto cleanup; \
    } while (0)
#define TWA_HTRY(expr)                                                    \
    do {                                                                  \
        hipError_t _e = (expr);                                           \
        if (_e != hipSuccess) {                                           \
            set_error(std::string(#expr) + ": " + hipGetErrorString(_e)); \
            rc = TWA_EHIP;                                                \
            goto cleanup;                                                 \
        }                                                                 \
    } while (0)

    {
        // memory check for the step store
        size_t freeb = 0, totb = 0;
        TWA_HTRY(hipMemGetInfo(&freeb, &totb));
        const double need = (double)plane * (3.0 * (K + 1) + 13.0 * K + 3.0 * nseg + 18.0) +
                            (double)partsz * (2.0 * K + 5 + nseg) + (double)g.C2 * KP * ge * 7.0 +
                            (double)g.P * 2 * KP * ge * 2.0;
        if (need > 0.9 * (double)freeb) {
            set_error("twa_adjoint: the checkpoint segment needs " + std::to_string(need / 1e9) +
                      " GB of device memory; reduce ckpt_every");
            rc = TWA_ENOMEM;
            goto cleanup;
        }
    }
    TWA_TRY(alloc_buffers(g, false, 0, J, b, st));
    TWA_TRY(dalloc0(&m.s, plane * 3 * (K + 1), st));
    TWA_TRY(dalloc0(&m.d, plane * 3 * K, st));
    TWA_TRY(dalloc0(&m.y1, plane * 2 * K, st));
    TWA_TRY(dalloc0(&m.y2, plane * 2 * K, st));
    TWA_TRY(dalloc0(&m.q, plane * 2 * K, st));
    TWA_TRY(dalloc0(&m.ya1, plane * 2 * K, st));
    TWA_TRY(dalloc0(&m.ya2, plane * 2 * K, st));
    TWA_TRY(dalloc0(&m.partS, partsz * (K + 1), st));
    TWA_TRY(dalloc0(&m.partP, partsz * K, st));
    TWA_TRY(dalloc0(&m.g, (size_t)2 * g.Bp * se * K, st));
    TWA_TRY(dalloc0(&m.ckpt, plane * 3 * nseg, st));
    TWA_TRY(dalloc0(&m.ckpt_part, partsz * nseg, st));
    TWA_TRY(dalloc0(&m.Aa, (size_t)g.P * 2 * KP * ge, st));
    TWA_TRY(dalloc0(&m.lam, plane * 6, st));
    TWA_TRY(dalloc0(&m.M1, plane * 6, st));
    TWA_TRY(dalloc0(&m.Rb, plane * 6, st));
    TWA_TRY(dalloc0(&m.nu2, (size_t)2 * g.C2 * KP * ge, st));
    TWA_TRY(dalloc0(&m.nu1, (size_t)2 * g.C2 * KP * ge, st));
    TWA_TRY(dalloc0(&m.nu2p, partsz * 2, st));
    TWA_TRY(dalloc0(&m.nu1p, partsz * 2, st));
    TWA_TRY(dalloc0((void**)&m.gacc, (size_t)4 * g.nmt * g.Bp * sizeof(double), st));
    TWA_HTRY(hipMalloc(&Wa, (size_t)N * N * sizeof(double)));
    TWA_HTRY(hipMalloc(&Fa, (size_t)N * N * sizeof(double)));
    TWA_TRY(dfactor_dalpha(pump, Wa, Fa, st));
    TWA_TRY(launch_build_A(g, pump->W, pump->F, dt, b.A, st));
    TWA_TRY(launch_build_A(g, Wa, Fa, dt, m.Aa, st));
    TWA_TRY(launch_init_state(g, b, c, nullptr, st));
    TWA_TRY(launch_reduce_state(g, b.s[0], b.part[0], st));
    TWA_HTRY(hipMemsetAsync(b.step, 0, sizeof(int64_t), st));
    TWA_HTRY(hipEventCreate(&e0));
    TWA_HTRY(hipEventCreate(&e1));
    TWA_HTRY(hipEventCreate(&e2));
    TWA_HTRY(hipEventRecord(e0, st));

    // ---------------- forward with checkpoints
    for (int64_t n = 0; n < n_steps; ++n) {
        if (n % K == 0) {
            // the state and its spin sums exactly as the forward holds them, so
            // that the recomputation reproduces the forward bit for bit
            TWA_HTRY(hipMemcpyAsync((char*)m.ckpt + (size_t)(n / K) * 3 * plane, b.s[cur], 3 * plane,
                                    hipMemcpyDeviceToDevice, st));
            TWA_HTRY(hipMemcpyAsync((char*)m.ckpt_part + (size_t)(n / K) * partsz, b.part[0], partsz,
                                    hipMemcpyDeviceToDevice, st));
        }
        TWA_TRY(launch_step_kernels(g, b, c, cur, false, nullptr, st));
        if (n + 1 > burnin) TWA_TRY(launch_observe(g, b, c, 1 - cur, false, st));
        cur = 1 - cur;
    }
    TWA_HTRY(hipEventRecord(e1, st));
    // spin-length drift and non-finite values of the forward run's last state
    TWA_TRY(launch_finish(g, b, cur, nblk_fin, st));
    hmom.resize((size_t)10 * g.Bp);
    hdiag.resize((size_t)2 * nblk_fin);
    {
        std::vector<S> tmp(hmom.size());
        TWA_HTRY(hipMemcpyAsync(tmp.data(), b.mom, tmp.size() * se, hipMemcpyDeviceToHost, st));
        TWA_HTRY(hipMemcpyAsync(hdiag.data(), b.diag, hdiag.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        TWA_HTRY(hipStreamSynchronize(st));
        for (size_t i = 0; i < tmp.size(); ++i) hmom[i] = (double)tmp[i];
        for (int i = 0; i < nblk_fin; ++i) {
            fwd_norm_dev = std::max(fwd_norm_dev, (double)hdiag[(size_t)i]);
            if (hdiag[(size_t)nblk_fin + i] != 0.f) fwd_nan = true;
        }
    }
    {
        const int64_t ns = n_steps - burnin;
        std::vector<double> traj((size_t)B * 5);
        for (int64_t k = 0; k < B; ++k)
            for (int q = 0; q < 5; ++q)
                traj[(size_t)k * 5 + q] =
                    ns > 0 ? (hmom[(size_t)(2 * q) * g.Bp + k] - hmom[(size_t)(2 * q + 1) * g.Bp + k]) / (double)ns
                           : NAN;
        std::memset(out, 0, sizeof(*out));
        out->I_gen = out->g2_gen = out->I_gen_se = out->g2_gen_se = NAN;
        finalize_moments(traj, B, out);
        out->n_samples = ns;
        out->step_criterion = std::max(p->gamma * (double)N, pump->lam_max) * dt;
        out->tile_config = cfg;
        out->max_norm_dev = fwd_norm_dev;
        out->nan_flag = fwd_nan ? 1 : 0;
        if (!std::isfinite(out->SpSm) || !std::isfinite(out->g2)) out->nan_flag = 1;
        if (ns <= 0) {
            set_error("twa_adjoint: empty averaging window");
            rc = TWA_EINVAL;
            goto cleanup;
        }
        // objective coefficients on the ensemble moments (T2, T3, T4, Z, ZZ)
        const double T2 = out->T2, T3 = out->T3, T4 = out->T4, Z = out->Z, ZZ = out->ZZ;
        const double den = T2 + 0.5 * Z;
        const double num = T4 + 2.0 * T3 - Z / 3.0 + 0.5 * ZZ - (4.0 / 3.0) * T2;
        const double a2 = 1.0 / (den * den), a3 = num / (den * den * den);
        const double c0[5] = {1.0, 0.0, 0.0, 0.5, 0.0};
        const double c1_[5] = {-(4.0 / 3.0) * a2 - 2.0 * a3, 2.0 * a2, a2, -a2 / 3.0 - a3, 0.5 * a2};
        // copies of the reverse sweep: both objectives, or the selected one in copy 0
        for (int q = 0; q < 5; ++q) {
            cf[0][q] = obj[0] == 0 ? c0[q] : c1_[q];
            cf[1][q] = nobj == 2 ? c1_[q] : 0.0;
        }
        scale = 1.0 / ((double)B * (double)ns);
    }

    // ---------------- backward
    TWA_TRY(src_init<PREC>(g, b.part[0], cf, scale, n_steps > burnin ? 1 : 0, m.lam, nobj, st));
    for (int64_t q = nseg - 1; q >= 0; --q) {
        const int64_t n0 = q * K, len = std::min<int64_t>(K, n_steps - n0);
        // recompute the segment from its checkpoint
        TWA_HTRY(hipMemcpyAsync(m.s, (char*)m.ckpt + (size_t)q * 3 * plane, 3 * plane, hipMemcpyDeviceToDevice, st));
        TWA_TRY(state_to_op<PREC>(g, m.s, b.Xop, st));
        TWA_HTRY(hipMemcpyAsync(m.partS, (char*)m.ckpt_part + (size_t)q * partsz, partsz, hipMemcpyDeviceToDevice,
                                st));
        hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(1), 0, st, b.step, n0);
        TWA_HTRY(hipGetLastError());
        for (int64_t j = 0; j < len; ++j) {
            char* sj = (char*)m.s + (size_t)j * 3 * plane;
            char* sj1 = (char*)m.s + (size_t)(j + 1) * 3 * plane;
            char* dj = (char*)m.d + (size_t)j * 3 * plane;
            char* y1j = (char*)m.y1 + (size_t)j * 2 * plane;
            char* y2j = (char*)m.y2 + (size_t)j * 2 * plane;
            char* qj = (char*)m.q + (size_t)j * 2 * plane;
            char* ya1j = (char*)m.ya1 + (size_t)j * 2 * plane;
            char* ya2j = (char*)m.ya2 + (size_t)j * 2 * plane;
            char* pSj = (char*)m.partS + (size_t)j * partsz;
            char* pSj1 = (char*)m.partS + (size_t)(j + 1) * partsz;
            char* pPj = (char*)m.partP + (size_t)j * partsz;
            char* gj = (char*)m.g + (size_t)j * 2 * g.Bp * se;
            EnsembleBuffers bj = b;
            bj.g = gj;
            TWA_TRY(launch_noise(g, bj, c, st));
            GemmCall p1;   // predictor, also storing its noise part Q = -sqrt(dt) F zeta (second K half)
            p1.kind = KIND_PRIMAL_WITH_Q; p1.stage = 1; p1.A = b.A; p1.X = b.Xop;
            p1.ldx = 2 * KP; p1.K = 2 * KP;
            p1.c1 = c.c1; p1.c2 = c.c2; p1.s_cur = sj; p1.dlt = dj; p1.Y = y1j; p1.Dop = b.Dop; p1.Sout = qj;
            p1.part_prim = pSj; p1.part_out = pPj; p1.g = gj; p1.step = b.step;
            TWA_TRY(launch_gemm_call(g, p1, st));
            GemmCall sa1;  // dY1/dalpha = A_alpha [s; zeta]
            sa1.kind = 2; sa1.stage = 1; sa1.A = m.Aa; sa1.X = b.Xop; sa1.ldx = 2 * KP;
            sa1.K = 2 * KP; sa1.Sout = ya1j; sa1.store_sign = 1.0;
            TWA_TRY(launch_gemm_call(g, sa1, st));
            GemmCall p2;
            p2.kind = 0; p2.stage = 2; p2.A = b.A; p2.X = b.Dop; p2.ldx = KP; p2.K = KP;
            p2.c1 = c.c1; p2.c2 = c.c2; p2.s_cur = sj; p2.s_next = sj1; p2.dlt = dj; p2.Y = y1j; p2.Y2out = y2j;
            p2.store_y2 = 1; p2.part_prim = pPj; p2.part_out = pSj1; p2.Xnext = b.Xop; p2.ldxn = 2 * KP; p2.g = gj;
            p2.step = b.step;
            TWA_TRY(launch_gemm_call(g, p2, st));
            GemmCall sa2;  // dY2/dalpha = dY1/dalpha + A_alpha,left D
            sa2.kind = 2; sa2.stage = 1; sa2.A = m.Aa; sa2.X = b.Dop; sa2.ldx = KP; sa2.K = KP;
            sa2.Sin = ya1j; sa2.Sout = ya2j; sa2.store_sign = 1.0;
            TWA_TRY(launch_gemm_call(g, sa2, st));
        }
        // reverse sweep through the segment
        for (int64_t j = len - 1; j >= 0; --j) {
            const int64_t n = n0 + j;
            char* sj = (char*)m.s + (size_t)j * 3 * plane;
            char* dj = (char*)m.d + (size_t)j * 3 * plane;
            char* y1j = (char*)m.y1 + (size_t)j * 2 * plane;
            char* y2j = (char*)m.y2 + (size_t)j * 2 * plane;
            char* qj = (char*)m.q + (size_t)j * 2 * plane;
            char* ya1j = (char*)m.ya1 + (size_t)j * 2 * plane;
            char* ya2j = (char*)m.ya2 + (size_t)j * 2 * plane;
            char* pSj = (char*)m.partS + (size_t)j * partsz;
            char* pPj = (char*)m.partP + (size_t)j * partsz;
            char* gj = (char*)m.g + (size_t)j * 2 * g.Bp * se;
            TWA_TRY(prep_nu2<PREC>(g, m.lam, sj, dj, m.nu2, m.nu2p, nobj, st));
            GemmCall a2;
            a2.kind = 3; a2.stage = 2; a2.ncopy = nobj; a2.A = b.A; a2.X = m.nu2; a2.ldx = KP;
            a2.x_copy = g.C2 * KP; a2.K = KP; a2.c1 = c.c1; a2.c2 = c.c2; a2.s_cur = sj; a2.dlt = dj; a2.Y = y1j;
            a2.Y2in = y2j; a2.Qin = qj; a2.YA = ya2j; a2.lam = m.lam; a2.M1 = m.M1; a2.Rb = m.Rb;
            a2.part_prim = pPj; a2.g = gj; a2.tpart_in = m.nu2p; a2.part_out = m.nu1p; a2.Xnext = m.nu1;
            a2.ldxn = KP; a2.gacc = m.gacc; a2.inv_w = 1.0 / pump->w;
            TWA_TRY(launch_gemm_call(g, a2, st));
            GemmCall a1;
            a1.kind = 4; a1.stage = 1; a1.ncopy = nobj; a1.A = b.A; a1.X = m.nu1; a1.ldx = KP;
            a1.x_copy = g.C2 * KP; a1.K = KP; a1.c1 = c.c1; a1.c2 = c.c2; a1.s_cur = sj; a1.Y = y1j; a1.Qin = qj;
            a1.YA = ya1j; a1.lam = m.lam; a1.M1 = m.M1; a1.Rb = m.Rb; a1.part_prim = pSj; a1.g = gj;
            a1.tpart_in = m.nu1p; a1.gacc = m.gacc; a1.inv_w = 1.0 / pump->w;
            std::memcpy(a1.srccoef, cf, sizeof(cf));
            a1.src_scale = scale;
            a1.src_on = n > burnin ? 1 : 0;   // the input state of step n is s_n
            TWA_TRY(launch_gemm_call(g, a1, st));
        }
    }
    TWA_HTRY(hipEventRecord(e2, st));
    hg.resize((size_t)4 * g.nmt * g.Bp);
    TWA_HTRY(hipMemcpyAsync(hg.data(), m.gacc, hg.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    TWA_HTRY(hipStreamSynchronize(st));
    TWA_HTRY(hipEventElapsedTime(&fwd_ms, e0, e1));
    TWA_HTRY(hipEventElapsedTime(&bwd_ms, e1, e2));
    for (int q = 0; q < 4; ++q) grads[q] = NAN;
    for (int cp = 0; cp < nobj; ++cp)
        for (int prm = 0; prm < 2; ++prm) {
            double s = 0;
            const size_t base = ((size_t)cp * 2 + prm) * g.nmt * g.Bp;
            for (size_t t = 0; t < (size_t)g.nmt * g.Bp; ++t) s += hg[base + t];
            grads[obj[cp] * 2 + prm] = s;
        }
    out->kernel_ms = fwd_ms + bwd_ms;
    out->adjoint_fwd_ms = fwd_ms;
    out->adjoint_bwd_ms = bwd_ms;
    for (int q = 0; q < 4; ++q)
        if (!std::isnan(grads[q]) && !std::isfinite(grads[q])) out->nan_flag = 1;
    rc = run_status("twa_adjoint", out->nan_flag != 0, out->max_norm_dev, p->norm_tol);
cleanup:
    if (rc != TWA_OK && rc != TWA_EUNSTABLE) hipStreamSynchronize(st);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e2) hipEventDestroy(e2);
    hipFree(Wa);
    hipFree(Fa);
    m.release();
    free_buffers(b);
    if (own) hipStreamDestroy(own);
#undef TWA_TRY
#undef TWA_HTRY
    return rc;
}

}  // namespace
}  // namespace twa

extern "C" TWA_API int twa_adjoint(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                                   int32_t ckpt_every, twa_observables* out, double* grads) {
    TWA_API_LOCK();
    using namespace twa;
    if (!p || !p->pump || !out || !grads || n_traj < 1 || n_steps < 1 || !(dt > 0) || !std::isfinite(dt) ||
        !(p->gamma > 0) || ckpt_every < 1) {
        set_error("twa_adjoint: need params with a pump, outputs, n_traj >= 1, n_steps >= 1, dt > 0, ckpt_every >= 1");
        return TWA_EINVAL;
    }
    if (!(p->pump->w > 0) || !std::isfinite(p->pump->alpha) || !p->pump->V || !p->pump->lam) {
        set_error("twa_adjoint: needs a pump from twa_build_pump with w > 0");
        return TWA_EINVAL;
    }
    if (p->integrator != TWA_INT_HEUN) {
        set_error("twa_adjoint: the reverse sweep is defined for the Heun integrator");
        return TWA_EINVAL;
    }
    if (p->adjoint_objectives < 0 || p->adjoint_objectives > 3) {
        set_error("twa_adjoint: adjoint_objectives is a mask of 1 (<S+S->) and 2 (g2), 0 = both");
        return TWA_EINVAL;
    }
    const int64_t burnin = p->burnin < 0 ? n_steps / 2 : p->burnin;
    if (burnin >= n_steps) {
        set_error("twa_adjoint: the averaging window is empty");
        return TWA_EINVAL;
    }
    const int K = (int)std::min<int64_t>(ckpt_every, n_steps);
    switch (p->precision) {
        case TWA_PREC_FP64: return adjoint_impl<TWA_PREC_FP64>(p, n_traj, dt, n_steps, seed, K, out, grads);
        case TWA_PREC_FP32: return adjoint_impl<TWA_PREC_FP32>(p, n_traj, dt, n_steps, seed, K, out, grads);
        case TWA_PREC_BF16X3: return adjoint_impl<TWA_PREC_BF16X3>(p, n_traj, dt, n_steps, seed, K, out, grads);
    }
    set_error("twa_adjoint: precision must be TWA_PREC_FP64, TWA_PREC_FP32 or TWA_PREC_BF16X3");
    return TWA_EINVAL;
}
