// Auxiliary kernels of the TWA trajectories: operand matrix, discrete
// initial sampling (SM Sec. S1 step 3), per-step noise draws (Eq. (S1)),
// time-averaged moments (SM Sec. S1 steps 5-6 and the closing remark on time
// averaging) and the two-time accumulation (Eq. (S3) and the response copies).
#include <algorithm>

#include "twa_internal.h"
#include "twa_device.h"

namespace twa {

template <int PREC>
struct P_ {
    typedef typename Prec<PREC>::G G;
    typedef typename Prec<PREC>::S S;
};

static inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// A = [-dt/2 W | -sqrt(dt) F], zero padded to P rows and 2P columns; in the
// split form 6P columns [Wh | Wh | Wl | Fh | Fh | Fl] against operand columns
// (sh, sl, sh, zh, zl, zh); stored stage-blocked (a_index) with kt columns
// per block
template <int PREC>
__global__ void build_A_kernel(const double* W, const double* F, int64_t N, int64_t P, int64_t kt, double cw,
                               double cf, typename Prec<PREC>::G* A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P * 2 * P) return;
    const int64_t i = t / (2 * P), j = t % (2 * P);
    double v = 0.0;
    if (i < N) {
        if (j < N) v = cw * W[i * N + j];
        else if (j >= P && j - P < N) v = cf * F[i * N + (j - P)];
    }
    if constexpr (Prec<PREC>::SPLIT == 3) {
        uint16_t hi, lo;
        bf16_split((float)v, hi, lo);
        const int64_t c = j < P ? j : 3 * P + (j - P);
        A[a_index(i, c, P, kt)].v = hi;
        A[a_index(i, c + P, P, kt)].v = hi;
        A[a_index(i, c + 2 * P, P, kt)].v = lo;
    } else {
        A[a_index(i, j, P, kt)] = Prec<PREC>::to_g((typename Prec<PREC>::S)v);
    }
}

template <int PREC>
static int build_A_t(const Geometry& g, const double* W, const double* F, double dt, void* A, hipStream_t st) {
    const int64_t n = g.P * 2 * g.P;
    hipLaunchKernelGGL(build_A_kernel<PREC>, dim3(nblocks(n, 256)), dim3(256), 0, st, W, F, g.N, g.P, g.kt,
                       -0.5 * dt, -sqrt(dt), static_cast<typename Prec<PREC>::G*>(A));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

#define TWA_DISPATCH(PRECV, CALL)                                  \
    switch (PRECV) {                                               \
        case TWA_PREC_FP64: { constexpr int PR = TWA_PREC_FP64; return CALL; } \
        case TWA_PREC_FP32: { constexpr int PR = TWA_PREC_FP32; return CALL; } \
        case TWA_PREC_BF16: { constexpr int PR = TWA_PREC_BF16; return CALL; } \
        case TWA_PREC_FP16: { constexpr int PR = TWA_PREC_FP16; return CALL; } \
        case TWA_PREC_BF16X3: { constexpr int PR = TWA_PREC_BF16X3; return CALL; } \
    }                                                              \
    set_error("unknown precision");                                \
    return TWA_EINVAL;

int launch_build_A(const Geometry& g, const double* W, const double* F, double dt, void* A, hipStream_t st) {
    TWA_DISPATCH(g.precision, (build_A_t<PR>(g, W, F, dt, A, st)))
}

// coherent exchange: A = [-dt/2 W | -sqrt(dt) F | dt Omega] against operand
// columns (s, zeta, s_perp), and the corrector's A2 = [-dt/2 W | dt Omega]
// against (D, D_perp), s_perp = (s^y, -s^x) for the (x, y) columns: the field
// of Eq. (S1) gains +dt (Omega s^y) in h^x and -dt (Omega s^x) in h^y; both
// stored stage-blocked (a_index)
template <int PREC>
__global__ void build_A_coh_kernel(const double* W, const double* F, const double* Om, int64_t N, int64_t P,
                                   int64_t kt, double cw, double cf, double co, typename Prec<PREC>::G* A,
                                   typename Prec<PREC>::G* A2) {
    typedef typename Prec<PREC>::S S;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P * 3 * P) return;
    const int64_t i = t / (3 * P), j = t % (3 * P);
    const int64_t blk = j / P, jj = j % P;
    double v = 0.0;
    if (i < N && jj < N) {
        const double m = blk == 0 ? W[i * N + jj] : blk == 1 ? F[i * N + jj] : Om[i * N + jj];
        v = (blk == 0 ? cw : blk == 1 ? cf : co) * m;
    }
    A[a_index(i, j, P, kt)] = Prec<PREC>::to_g((S)v);
    if (blk != 1) A2[a_index(i, blk == 0 ? jj : P + jj, P, kt)] = Prec<PREC>::to_g((S)v);
}

template <int PREC>
static int build_A_coh_t(const Geometry& g, const double* W, const double* F, const double* Om, double dt, void* A,
                         void* A2, hipStream_t st) {
    if constexpr (Prec<PREC>::SPLIT != 1) {
        set_error("coherent exchange: not with the split precision");
        return TWA_EINVAL;
    } else {
        const int64_t n = g.P * 3 * g.P;
        hipLaunchKernelGGL(build_A_coh_kernel<PREC>, dim3(nblocks(n, 256)), dim3(256), 0, st, W, F, Om, g.N, g.P,
                           g.kt, -0.5 * dt, -sqrt(dt), dt, static_cast<typename Prec<PREC>::G*>(A),
                           static_cast<typename Prec<PREC>::G*>(A2));
        TWA_HIP_CHECK(hipGetLastError());
        return TWA_OK;
    }
}

int launch_build_A_coh(const Geometry& g, const double* W, const double* F, const double* Om, double dt, void* A,
                       void* A2, hipStream_t st) {
    TWA_DISPATCH(g.precision, (build_A_coh_t<PR>(g, W, F, Om, dt, A, A2, st)))
}

// ---------------------------------------------------------------------------
// discrete initial sampling: s^{x,y} = +-1 from Philox bits, s^z = s0z
template <int PREC>
__global__ void init_kernel(int64_t N, int64_t B, int64_t P, int64_t Bp, double s0z, uint32_t k0, uint32_t k1,
                            uint32_t point, const double* init, typename Prec<PREC>::S* s,
                            typename Prec<PREC>::S* norm0, typename Prec<PREC>::G* Xop, int coh) {
    typedef typename Prec<PREC>::S S;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bp * P) return;
    const int64_t k = t / P, i = t % P;
    S x = 0, y = 0, z = 0;
    if (k < B && i < N) {
        if (init) {
            x = (S)init[(0 * B + k) * N + i];
            y = (S)init[(1 * B + k) * N + i];
            z = (S)init[(2 * B + k) * N + i];
        } else {
            const uint32_t m = (uint32_t)(i >> 6), j = (uint32_t)(i & 63);
            const U4 w = philox4x32_10(U4{m, (uint32_t)k, 0u, TAG_INIT | (point << 8)}, k0, k1);
            const uint32_t words[4] = {w.x, w.y, w.z, w.w};
            const uint32_t bx = 2 * j, by = 2 * j + 1;
            x = ((words[bx >> 5] >> (bx & 31)) & 1u) ? S(1) : S(-1);
            y = ((words[by >> 5] >> (by & 31)) & 1u) ? S(1) : S(-1);
            z = (S)s0z;
        }
    }
    const int64_t SP = Bp * P;
    s[t] = x;
    s[SP + t] = y;
    s[2 * SP + t] = z;
    norm0[t] = x * x + y * y + z * z;
    constexpr int SPL = Prec<PREC>::SPLIT;
    const int64_t ld = (2 + coh) * P * SPL;   // operand column length
    put_op<PREC>(Xop + opcol(k, 0) * ld + i, P, x);
    put_op<PREC>(Xop + opcol(k, 1) * ld + i, P, y);
    if (coh) {   // s_perp block: (s^y, -s^x)
        Xop[opcol(k, 0) * ld + 2 * P + i] = Prec<PREC>::to_g(y);
        Xop[opcol(k, 1) * ld + 2 * P + i] = Prec<PREC>::to_g(-x);
    }
}

template <int PREC>
static int init_t(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const double* init,
                  hipStream_t st) {
    typedef typename Prec<PREC>::S S;
    typedef typename Prec<PREC>::G G;
    const int64_t n = g.Bp * g.P;
    hipLaunchKernelGGL(init_kernel<PREC>, dim3(nblocks(n, 256)), dim3(256), 0, st, g.N, g.B, g.P, g.Bp, c.s0z,
                       c.key0, c.key1, (uint32_t)c.point, init, static_cast<S*>(b.s[0]), static_cast<S*>(b.norm0),
                       static_cast<G*>(b.Xop), g.coh);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

int launch_init_state(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const double* init,
                      hipStream_t st) {
    TWA_DISPATCH(g.precision, (init_t<PR>(g, b, c, init, st)))
}

// partial spin sums of a state over M tiles: part[c][mt][k]
template <typename S>
__global__ void reduce_state_kernel(const S* s, int64_t P, int64_t Bp, int64_t nmt, int64_t mtile, S* part) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nmt * Bp) return;
    const int64_t c = t / (nmt * Bp), r = t % (nmt * Bp), q = r / Bp, k = r % Bp;
    const S* row = s + c * Bp * P + k * P + q * mtile;
    S acc = 0;
    for (int64_t i = 0; i < mtile; ++i) acc += row[i];
    part[t] = acc;
}

int launch_reduce_state(const Geometry& g, const void* s, void* part, hipStream_t st) {
    const int64_t n = 3 * g.nmt * g.Bp;
    const int64_t mtile = g.P / g.nmt;
    if (g.precision == TWA_PREC_FP64)
        hipLaunchKernelGGL(reduce_state_kernel<double>, dim3(nblocks(n, 256)), dim3(256), 0, st,
                           static_cast<const double*>(s), g.P, g.Bp, g.nmt, mtile, static_cast<double*>(part));
    else
        hipLaunchKernelGGL(reduce_state_kernel<float>, dim3(nblocks(n, 256)), dim3(256), 0, st,
                           static_cast<const float*>(s), g.P, g.Bp, g.nmt, mtile, static_cast<float*>(part));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

// ---------------------------------------------------------------------------
// per-step noise: zeta^{x,y} of every (trajectory, spin) into the operand,
// g^{x,y} of every trajectory.  The step index is read from device memory.
template <int PREC>
__global__ void noise_kernel(int64_t N, int64_t B, int64_t P, int64_t Bp, uint32_t k0, uint32_t k1,
                             uint32_t point, const int64_t* step, typename Prec<PREC>::G* Xop,
                             typename Prec<PREC>::S* g, int64_t ldop) {
    typedef typename Prec<PREC>::S S;
    // grid: x over Philox slots (pairs of spins), y over trajectories (strided)
    const int64_t nslot = (N + 1) / 2;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nslot) return;
    const uint32_t n = (uint32_t)step[0];
    for (int64_t k = blockIdx.y; k < B; k += gridDim.y) {
        const U4 w = philox4x32_10(U4{(uint32_t)m, (uint32_t)k, n, TAG_PUMP | (point << 8)}, k0, k1);
        S z0, z1, z2, z3;
        box_muller(w.x, w.y, z0, z1);
        box_muller(w.z, w.w, z2, z3);
        const int64_t i = 2 * m;
        constexpr int SPL = Prec<PREC>::SPLIT;
        typename Prec<PREC>::G* cx = Xop + opcol(k, 0) * ldop + P * SPL;
        typename Prec<PREC>::G* cy = Xop + opcol(k, 1) * ldop + P * SPL;
        put_op<PREC>(cx + i, P, z0);
        put_op<PREC>(cy + i, P, z1);
        if (i + 1 < N) {
            put_op<PREC>(cx + i + 1, P, z2);
            put_op<PREC>(cy + i + 1, P, z3);
        }
        if (m == 0) {
            const U4 v = philox4x32_10(U4{0u, (uint32_t)k, n, TAG_COLLECTIVE | (point << 8)}, k0, k1);
            S g0, g1;
            box_muller(v.x, v.y, g0, g1);
            g[k] = g0;
            g[Bp + k] = g1;
        }
    }
}

template <int PREC>
static int noise_t(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, hipStream_t st) {
    const int64_t nslot = (g.N + 1) / 2;
    hipLaunchKernelGGL(noise_kernel<PREC>, dim3(nblocks(nslot, 256), (unsigned)std::min<int64_t>(g.B, 65535)),
                       dim3(256), 0, st, g.N, g.B, g.P,
                       g.Bp, c.key0,
                       c.key1, (uint32_t)c.point, (const int64_t*)b.step,
                       static_cast<typename Prec<PREC>::G*>(b.Xop), static_cast<typename Prec<PREC>::S*>(b.g),
                       (int64_t)(2 + g.coh) * g.P * Prec<PREC>::SPLIT);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

int launch_noise(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, hipStream_t st) {
    TWA_DISPATCH(g.precision, (noise_t<PR>(g, b, c, st)))
}

// ---------------------------------------------------------------------------
// response copies at the origin: ds = x^ (copy 0) and ds = y^ (copy 1)
template <int PREC>
__global__ void seed_kernel(int64_t N, int64_t B, int64_t P, int64_t Bp, int64_t C2, typename Prec<PREC>::S* ts,
                            typename Prec<PREC>::G* tXop) {
    typedef typename Prec<PREC>::S S;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bp * P) return;
    const int64_t k = t / P, i = t % P;
    const S one = (k < B && i < N) ? S(1) : S(0);
    const int64_t SP = Bp * P;
    for (int cp = 0; cp < 2; ++cp) {
        S* base = ts + cp * 3 * SP;
        base[t] = cp == 0 ? one : S(0);
        base[SP + t] = cp == 1 ? one : S(0);
        base[2 * SP + t] = S(0);
        // operand columns of pitch P (split form: hi, lo, hi blocks of P)
        constexpr int SPL = Prec<PREC>::SPLIT;
        typename Prec<PREC>::G* op = tXop + cp * C2 * P * SPL;
        put_op<PREC>(op + opcol(k, 0) * P * SPL + i, P, cp == 0 ? one : S(0));
        put_op<PREC>(op + opcol(k, 1) * P * SPL + i, P, cp == 1 ? one : S(0));
    }
}

template <int PREC>
static int seed_t(const Geometry& g, const EnsembleBuffers& b, int cur, hipStream_t st) {
    typedef typename Prec<PREC>::S S;
    const int64_t n = g.Bp * g.P;
    hipLaunchKernelGGL(seed_kernel<PREC>, dim3(nblocks(n, 256)), dim3(256), 0, st, g.N, g.B, g.P, g.Bp, g.C2,
                       static_cast<S*>(b.ts[cur]), static_cast<typename Prec<PREC>::G*>(b.tXop));
    TWA_HIP_CHECK(hipGetLastError());
    for (int cp = 0; cp < 2; ++cp) {
        int rc = launch_reduce_state(g, static_cast<S*>(b.ts[cur]) + cp * 3 * g.Bp * g.P,
                                     static_cast<S*>(b.tpart[0]) + cp * 3 * g.nmt * g.Bp, st);
        if (rc) return rc;
    }
    return TWA_OK;
}

int launch_seed_tangents(const Geometry& g, const EnsembleBuffers& b, int cur, hipStream_t st) {
    TWA_DISPATCH(g.precision, (seed_t<PR>(g, b, cur, st)))
}

// ---------------------------------------------------------------------------
// observation after a step: window moments (Kahan-compensated time sums per
// trajectory), the two-time origin and lag sums per jackknife block.
template <typename S>
__device__ __forceinline__ void kahan_add(S* sum, S* comp, S v) {
    const S s = *sum, c = *comp;
    const S y = v - c;
    const S t = s + y;
    *comp = (t - s) - y;
    *sum = t;
}

template <typename S>
__global__ __launch_bounds__(256) void observe_kernel(int64_t B, int64_t Bp, int64_t nmt, int J, int64_t burnin,
                                                      int64_t stride, int64_t L, const int64_t* step, const S* part,
                                                      const S* tpart, int64_t tpart_copy, int tangents, S* mom,
                                                      S* sm0, double* lag) {
    __shared__ double red[6][256];
    const int64_t kst = step[0];
    const int j = blockIdx.x;
    const int64_t klo = ((int64_t)j * B + J - 1) / J, khi = ((int64_t)(j + 1) * B + J - 1) / J;
    const bool in_window = kst > burnin;
    const bool origin = L > 0 && kst == burnin;
    int64_t l = -1;
    if (L > 0 && kst >= burnin && (kst - burnin) % stride == 0 && (kst - burnin) / stride < L)
        l = (kst - burnin) / stride;
    double acc6[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = klo + threadIdx.x; k < khi; k += blockDim.x) {
        S sxyz[3];
        tile_sums<S, 3>(part, nmt, Bp, k, 0, sxyz);
        const S Sx = sxyz[0], Sy = sxyz[1], Sz = sxyz[2];
        if (in_window) {
            const S T2 = S(0.25) * (Sx * Sx + Sy * Sy);
            const S v[5] = {T2, T2 * Sz, T2 * T2, Sz, Sz * Sz};
#pragma unroll
            for (int m = 0; m < 5; ++m) kahan_add(mom + (2 * m) * Bp + k, mom + (2 * m + 1) * Bp + k, v[m]);
        }
        if (origin) {
            sm0[k] = Sx;
            sm0[Bp + k] = Sy;
        }
        if (l >= 0) {
            const double x0 = (double)sm0[k], y0 = (double)sm0[Bp + k];
            acc6[0] += 0.25 * ((double)Sx * x0 + (double)Sy * y0);
            acc6[1] += 0.25 * ((double)Sy * x0 - (double)Sx * y0);
            if (tangents) {
                for (int cp = 0; cp < 2; ++cp) {
                    S txy[2];
                    tile_sums<S, 2>(tpart + cp * tpart_copy, nmt, Bp, k, 0, txy);
                    acc6[2 + 2 * cp] += (double)txy[0];
                    acc6[3 + 2 * cp] += (double)txy[1];
                }
            }
        }
    }
    if (l < 0) return;   // uniform across the block
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc6[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) lag[(l * J + j) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

int launch_observe(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int cur, bool tangents,
                   hipStream_t st) {
    (void)cur;
    const int64_t tcopy = 3 * g.nmt * g.Bp;
    if (g.precision == TWA_PREC_FP64)
        hipLaunchKernelGGL(observe_kernel<double>, dim3(c.J), dim3(256), 0, st, g.B, g.Bp, g.nmt, c.J, c.burnin,
                           c.lag_stride, c.n_lags, (const int64_t*)b.step, static_cast<const double*>(b.part[0]),
                           static_cast<const double*>(b.tpart[0]), tcopy, tangents ? 1 : 0,
                           static_cast<double*>(b.mom), static_cast<double*>(b.sm0), b.lag);
    else
        hipLaunchKernelGGL(observe_kernel<float>, dim3(c.J), dim3(256), 0, st, g.B, g.Bp, g.nmt, c.J, c.burnin,
                           c.lag_stride, c.n_lags, (const int64_t*)b.step, static_cast<const float*>(b.part[0]),
                           static_cast<const float*>(b.tpart[0]), tcopy, tangents ? 1 : 0,
                           static_cast<float*>(b.mom), static_cast<float*>(b.sm0), b.lag);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

// ---------------------------------------------------------------------------
// end-of-run diagnostics: max | |s|^2 - |s0|^2 | and non-finite flag per block
template <typename S>
__global__ __launch_bounds__(256) void finish_kernel(const S* s, const S* norm0, int64_t N, int64_t B, int64_t P,
                                                     int64_t Bp, float* diag) {
    __shared__ float rmax[256];
    __shared__ int rnan[256];
    float m = 0.f;
    int bad = 0;
    const int64_t SP = Bp * P;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < B * N; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / N, i = t % N, o = k * P + i;
        const S x = s[o], y = s[SP + o], z = s[2 * SP + o];
        const S d = x * x + y * y + z * z - norm0[o];
        if (!isfinite((double)d)) bad = 1;
        else m = fmaxf(m, (float)fabs((double)d));
    }
    rmax[threadIdx.x] = m;
    rnan[threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rmax[threadIdx.x] = fmaxf(rmax[threadIdx.x], rmax[threadIdx.x + w]);
            rnan[threadIdx.x] |= rnan[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        diag[blockIdx.x] = rmax[0];
        diag[gridDim.x + blockIdx.x] = (float)rnan[0];
    }
}

int launch_finish(const Geometry& g, const EnsembleBuffers& b, int cur, int nblk, hipStream_t st) {
    if (g.precision == TWA_PREC_FP64)
        hipLaunchKernelGGL(finish_kernel<double>, dim3(nblk), dim3(256), 0, st, static_cast<const double*>(b.s[cur]),
                           static_cast<const double*>(b.norm0), g.N, g.B, g.P, g.Bp, b.diag);
    else
        hipLaunchKernelGGL(finish_kernel<float>, dim3(nblk), dim3(256), 0, st, static_cast<const float*>(b.s[cur]),
                           static_cast<const float*>(b.norm0), g.N, g.B, g.P, g.Bp, b.diag);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <typename S>
__global__ void export_kernel(const S* s, int64_t N, int64_t B, int64_t P, int64_t Bp, double* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * B * N) return;
    const int64_t c = t / (B * N), r = t % (B * N), k = r / N, i = r % N;
    out[t] = (double)s[c * Bp * P + k * P + i];
}

int launch_export_state(const Geometry& g, const void* s, double* out, hipStream_t st) {
    const int64_t n = 3 * g.B * g.N;
    if (g.precision == TWA_PREC_FP64)
        hipLaunchKernelGGL(export_kernel<double>, dim3(nblocks(n, 256)), dim3(256), 0, st,
                           static_cast<const double*>(s), g.N, g.B, g.P, g.Bp, out);
    else
        hipLaunchKernelGGL(export_kernel<float>, dim3(nblocks(n, 256)), dim3(256), 0, st,
                           static_cast<const float*>(s), g.N, g.B, g.P, g.Bp, out);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

// ---------------------------------------------------------------------------
// kernel-level entry points for the parity tests
__global__ void philox_kernel(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const U4 r = philox4x32_10(U4{ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3]}, k0, k1);
    out[4 * t] = r.x;
    out[4 * t + 1] = r.y;
    out[4 * t + 2] = r.z;
    out[4 * t + 3] = r.w;
}

int launch_philox(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t st) {
    if (n <= 0) return TWA_OK;
    hipLaunchKernelGGL(philox_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, ctr, n, k0, k1, out);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <typename S>
__global__ void noise_debug_kernel(uint32_t k0, uint32_t k1, uint32_t step, uint32_t point, int64_t B, int64_t N,
                                   double* zeta, double* g) {
    const int64_t nslot = (N + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * nslot) return;
    const int64_t k = t / nslot, m = t % nslot;
    const U4 w = philox4x32_10(U4{(uint32_t)m, (uint32_t)k, step, TAG_PUMP | (point << 8)}, k0, k1);
    S z0, z1, z2, z3;
    box_muller(w.x, w.y, z0, z1);
    box_muller(w.z, w.w, z2, z3);
    const int64_t i = 2 * m;
    zeta[k * N + i] = (double)z0;
    zeta[B * N + k * N + i] = (double)z1;
    if (i + 1 < N) {
        zeta[k * N + i + 1] = (double)z2;
        zeta[B * N + k * N + i + 1] = (double)z3;
    }
    if (m == 0) {
        const U4 v = philox4x32_10(U4{0u, (uint32_t)k, step, TAG_COLLECTIVE | (point << 8)}, k0, k1);
        S g0, g1;
        box_muller(v.x, v.y, g0, g1);
        g[k] = (double)g0;
        g[B + k] = (double)g1;
    }
}

int launch_noise_debug(uint64_t seed, int64_t step, int32_t point, int64_t B, int64_t N, int fp64, double* zeta,
                       double* g, hipStream_t st) {
    const int64_t n = B * ((N + 1) / 2);
    if (n <= 0) return TWA_OK;
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    if (fp64)
        hipLaunchKernelGGL(noise_debug_kernel<double>, dim3(nblocks(n, 256)), dim3(256), 0, st, k0, k1,
                           (uint32_t)step, (uint32_t)point, B, N, zeta, g);
    else
        hipLaunchKernelGGL(noise_debug_kernel<float>, dim3(nblocks(n, 256)), dim3(256), 0, st, k0, k1,
                           (uint32_t)step, (uint32_t)point, B, N, zeta, g);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

}  // namespace twa
