// Fused small-N path of the TWA trajectories (Eq. (S1), SM Sec. S1): for
// short chains the per-step work is a few N x N matrix-vector products per
// trajectory, far too little to fill the device per launch, so the run is
// bound by per-step latency.  One launch integrates every step: a trajectory
// occupies NL = 2^k >= N lanes of one wave (lane i holds spin i), the scaled
// operand rows [-dt/2 W | -sqrt(dt) F] live in LDS, the spin vectors of each
// trajectory are exchanged through LDS, every step's noise is drawn in
// registers from the same Philox counters as the multi-kernel path, and the
// window moments are Kahan-summed in registers.  Heun and the semi-implicit
// midpoint scheme; FP64 or FP32 arithmetic.
#include <algorithm>
#include <cmath>

#include "twa_device.h"
#include "twa_internal.h"

namespace twa {
namespace {

constexpr int SMALL_NMAX = 64;
constexpr int SMALL_THREADS = 256;

template <typename S>
__device__ __forceinline__ void kahan(S& sum, S& comp, S v) {
    const S y = v - comp;
    const S t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// midpoint rotation of the semi-implicit scheme (same closed form as the step kernels)
template <typename S>
__device__ __forceinline__ void rotate(S x, S y, S z, S Hx, S Hy, S& ox, S& oy, S& oz) {
    const S bx = S(0.5) * Hy, by = S(-0.5) * Hx;
    const S ax = x - by * z, ay = y + bx * z, az = z - (bx * y - by * x);
    const S bd = bx * ax + by * ay;
    const S inv = S(1) / (S(1) + bx * bx + by * by);
    ox = (ax - by * az + bx * bd) * inv;
    oy = (ay + bx * az + by * bd) * inv;
    oz = (az - (bx * ay - by * ax)) * inv;
}

template <typename S, int NL>
__global__ __launch_bounds__(SMALL_THREADS) void small_run_kernel(
    int64_t N, int64_t B, int64_t P, int64_t Bp, const double* __restrict__ W, const double* __restrict__ F,
    double cw, double cf, S c1, S c2, uint32_t k0, uint32_t k1, uint32_t point, int64_t n_steps, int64_t burnin,
    int sib, const S* __restrict__ s_in, S* __restrict__ s_out, S* __restrict__ mom) {
    constexpr int TPW = 64 / NL;                       // trajectories per wave
    constexpr int TPB = TPW * (SMALL_THREADS / 64);    // trajectories per block
    __shared__ S Aw[SMALL_NMAX * SMALL_NMAX];          // -dt/2 W, row-major N x N
    __shared__ S Af[SMALL_NMAX * SMALL_NMAX];          // -sqrt(dt) F
    __shared__ S vx[TPB][NL], vy[TPB][NL], ux[TPB][NL], uy[TPB][NL];
    const int n = (int)N;
    for (int t = threadIdx.x; t < n * n; t += SMALL_THREADS) {
        Aw[t] = (S)(cw * W[t]);
        Af[t] = (S)(cf * F[t]);
    }
    const int tl = threadIdx.x / NL, i = threadIdx.x % NL;   // trajectory in block, spin
    const int64_t k = (int64_t)blockIdx.x * TPB + tl;
    const bool live = k < B && i < n;
    const int64_t SP = Bp * P;
    S x = 0, y = 0, z = 0;
    if (live) {
        x = s_in[k * P + i];
        y = s_in[SP + k * P + i];
        z = s_in[2 * SP + k * P + i];
    }
    S msum[5] = {0, 0, 0, 0, 0}, mcmp[5] = {0, 0, 0, 0, 0};
    const S* aw = Aw + i * n;
    const S* af = Af + i * n;
    __syncthreads();

    for (int64_t st = 0; st < n_steps; ++st) {
        // noise of the step (counters of the multi-kernel path)
        S zx = 0, zy = 0, g0 = 0, g1 = 0;
        {
            const uint32_t ks = (uint32_t)k, ns = (uint32_t)st;
            const U4 w = philox4x32_10(U4{(uint32_t)(i >> 1), ks, ns, TAG_PUMP | (point << 8)}, k0, k1);
            S a0, a1, a2, a3;
            box_muller(w.x, w.y, a0, a1);
            box_muller(w.z, w.w, a2, a3);
            if (live) {
                zx = (i & 1) ? a2 : a0;
                zy = (i & 1) ? a3 : a1;
            }
            const U4 v = philox4x32_10(U4{0u, ks, ns, TAG_COLLECTIVE | (point << 8)}, k0, k1);
            box_muller(v.x, v.y, g0, g1);
        }
        // stage 1: fields at s_n
        vx[tl][i] = x;
        vy[tl][i] = y;
        ux[tl][i] = zx;
        uy[tl][i] = zy;
        __syncthreads();
        S Yx = 0, Yy = 0, Qx = 0, Qy = 0, Sx = 0, Sy = 0;
        for (int j = 0; j < n; ++j) {
            Yx += aw[j] * vx[tl][j];
            Yy += aw[j] * vy[tl][j];
            Qx += af[j] * ux[tl][j];
            Qy += af[j] * uy[tl][j];
            Sx += vx[tl][j];
            Sy += vy[tl][j];
        }
        const S Hx = (Yx + Qx) + (c1 * Sx + c2 * g0), Hy = (Yy + Qy) + (c1 * Sy + c2 * g1);
        S px, py, pz, dx = 0, dy = 0, dz = 0;
        if (sib) {
            rotate(x, y, z, Hx, Hy, px, py, pz);
        } else {
            dx = z * Hx;
            dy = z * Hy;
            dz = -(x * Hx + y * Hy);
            px = x + dx;
            py = y + dy;
            pz = z + dz;
        }
        if (!live) px = py = pz = 0;
        // stage 2: fields at the predictor (Heun) or the midpoint (semi-implicit)
        const S mx = sib ? S(0.5) * (x + px) : px, my = sib ? S(0.5) * (y + py) : py;
        __syncthreads();   // stage-1 reads done
        vx[tl][i] = mx;
        vy[tl][i] = my;
        __syncthreads();
        S Y2x = 0, Y2y = 0, S2x = 0, S2y = 0;
        for (int j = 0; j < n; ++j) {
            Y2x += aw[j] * vx[tl][j];
            Y2y += aw[j] * vy[tl][j];
            S2x += vx[tl][j];
            S2y += vy[tl][j];
        }
        const S H2x = (Y2x + Qx) + (c1 * S2x + c2 * g0), H2y = (Y2y + Qy) + (c1 * S2y + c2 * g1);
        if (sib) {
            rotate(x, y, z, H2x, H2y, x, y, z);
        } else {
            const S ex = pz * H2x, ey = pz * H2y, ez = -(px * H2x + py * H2y);
            x = x + S(0.5) * (dx + ex);
            y = y + S(0.5) * (dy + ey);
            z = z + S(0.5) * (dz + ez);
        }
        if (!live) x = y = z = 0;
        // window moments of the new state
        if (st + 1 > burnin) {
            __syncthreads();   // stage-2 reads done
            vx[tl][i] = x;
            vy[tl][i] = y;
            ux[tl][i] = z;
            __syncthreads();
            if (i == 0) {
                S Tx = 0, Ty = 0, Tz = 0;
                for (int j = 0; j < n; ++j) {
                    Tx += vx[tl][j];
                    Ty += vy[tl][j];
                    Tz += ux[tl][j];
                }
                const S T2 = S(0.25) * (Tx * Tx + Ty * Ty);
                const S v[5] = {T2, T2 * Tz, T2 * T2, Tz, Tz * Tz};
#pragma unroll
                for (int m = 0; m < 5; ++m) kahan(msum[m], mcmp[m], v[m]);
            }
        }
        __syncthreads();   // all reads of this step done before the next step's writes
    }
    if (k < B) {
        if (i < n) {
            s_out[k * P + i] = x;
            s_out[SP + k * P + i] = y;
            s_out[2 * SP + k * P + i] = z;
        }
        if (i == 0)
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                mom[(2 * m) * Bp + k] = msum[m];
                mom[(2 * m + 1) * Bp + k] = mcmp[m];
            }
    }
}

template <typename S, int NL>
int launch_small_t(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const twa_pump* pump, double dt,
                   int64_t n_steps, int sib, int out_cur, hipStream_t st) {
    constexpr int TPB = (64 / NL) * (SMALL_THREADS / 64);
    const unsigned grid = (unsigned)((g.B + TPB - 1) / TPB);
    hipLaunchKernelGGL((small_run_kernel<S, NL>), dim3(grid), dim3(SMALL_THREADS), 0, st, g.N, g.B, g.P, g.Bp, pump->W,
                       pump->F, -0.5 * dt, -std::sqrt(dt), (S)c.c1, (S)c.c2, c.key0, c.key1, (uint32_t)c.point,
                       n_steps, c.burnin, sib, static_cast<const S*>(b.s[0]), static_cast<S*>(b.s[out_cur]),
                       static_cast<S*>(b.mom));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <typename S>
int launch_small_s(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const twa_pump* pump, double dt,
                   int64_t n_steps, int sib, int out_cur, hipStream_t st) {
    if (g.N <= 8) return launch_small_t<S, 8>(g, b, c, pump, dt, n_steps, sib, out_cur, st);
    if (g.N <= 16) return launch_small_t<S, 16>(g, b, c, pump, dt, n_steps, sib, out_cur, st);
    if (g.N <= 32) return launch_small_t<S, 32>(g, b, c, pump, dt, n_steps, sib, out_cur, st);
    return launch_small_t<S, 64>(g, b, c, pump, dt, n_steps, sib, out_cur, st);
}

}  // namespace

bool small_path_applies(int precision, int64_t N, int64_t n_lags) {
    return N <= SMALL_NMAX && n_lags == 0 && (precision == TWA_PREC_FP64 || precision == TWA_PREC_FP32);
}

int launch_small_run(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const twa_pump* pump,
                     double dt, int64_t n_steps, int out_cur, hipStream_t st) {
    if (g.N > SMALL_NMAX) {
        set_error("fused small-N path: N > 64");
        return TWA_EINVAL;
    }
    const int sib = g.integrator == TWA_INT_SIB ? 1 : 0;
    if (g.precision == TWA_PREC_FP64) return launch_small_s<double>(g, b, c, pump, dt, n_steps, sib, out_cur, st);
    if (g.precision == TWA_PREC_FP32) return launch_small_s<float>(g, b, c, pump, dt, n_steps, sib, out_cur, st);
    set_error("fused small-N path: FP64 or FP32 only");
    return TWA_EINVAL;
}

}  // namespace twa
