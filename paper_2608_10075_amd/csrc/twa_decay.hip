// Correlated decay: a symmetric PSD decay matrix G_ij in place of the
// collective decay Gamma (the general-matrix model the paper's Perspectives
// name).  The step needs no kernel of its own: with the drift matrix W - G
// and the noise factor sqrt(W + G) in the operand and the collective terms
// switched off, the stage kernels integrate Eq. (S1) with the collective sum
// Gamma S^a replaced by sum_j G_ij s^a_j (the decay and pump noises are
// independent Gaussians, so together they are one Gaussian of covariance
// (W + G) dt).  What is new is the estimator of correlated emission, SM
// Sec. S1 step 6: per observed state it needs G s^x, G s^y (a contraction
// over the state part of the next step's operand), (G o G) s^z (a contraction
// over a packed z operand) and a per-trajectory reduction to nine scalars,
// which are Kahan-summed over the window:
//   E2 = sum_ab G_ab s+_a s-_b,  D = sum_a G_aa z_a,
//   Q3 = sum_b z_b |(G s+)_b|^2,  R = sum_a G_aa^2 z_a,  U = z^T (G o G) z,
//   V = Re sum_ab G_aa G_ab s+_a s-_b,
// accumulated as (E2, E2^2, E2 D, Q3, R, D^2, U, V, D).
#include "twa_device.h"
#include "twa_internal.h"

namespace twa {
namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// observation operands: G and G o G zero padded to P x P in the contraction
// type, stored stage-blocked (a_index), and the diagonal of G in the state type
template <int PREC>
__global__ void decay_ops_kernel(const double* G, int64_t N, int64_t P, int64_t kt, typename Prec<PREC>::G* AG,
                                 typename Prec<PREC>::G* AGG, typename Prec<PREC>::S* dg) {
    typedef typename Prec<PREC>::S S;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P * P) return;
    const int64_t i = t / P, j = t % P;
    const double v = (i < N && j < N) ? G[i * N + j] : 0.0;
    AG[a_index(i, j, P, kt)] = Prec<PREC>::to_g((S)v);
    AGG[a_index(i, j, P, kt)] = Prec<PREC>::to_g((S)(v * v));
    if (i == j) dg[i] = (S)v;
}

// z planes of all Bp trajectories as the operand of a contraction over Bp / 2
// column pairs: trajectory k sits in column (k mod Bp/2, k div Bp/2), so the
// store kind writes (G o G) z_k to plane k div Bp/2, row k mod Bp/2 of an
// output with Bp/2 rows per plane, i.e. to k * P in a plain [Bp][P] layout
template <int PREC>
__global__ void pack_z_kernel(const typename Prec<PREC>::S* s, int64_t Bp, int64_t P, typename Prec<PREC>::G* Zop) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bp * P) return;
    const int64_t k = t / P, i = t % P, half = Bp / 2;
    Zop[opcol(k % half, (int)(k / half)) * P + i] = Prec<PREC>::to_g(s[2 * Bp * P + t]);
}

__device__ __forceinline__ void kahan_add(double& sum, double& comp, double v) {
    const double y = v - comp;
    const double t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// one block per trajectory: the nine estimator quantities of the state, in a
// fixed summation order (FP64 accumulation), added to the window sums
template <typename S>
__global__ __launch_bounds__(256) void decay_reduce_kernel(const S* __restrict__ s, const S* __restrict__ GX,
                                                           const S* __restrict__ UZ, const S* __restrict__ dg,
                                                           int64_t N, int64_t P, int64_t Bp,
                                                           double* __restrict__ gmom) {
    __shared__ double red[6][256];
    const int64_t k = blockIdx.x;
    const int64_t SP = Bp * P, o = k * P;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
    for (int64_t i = threadIdx.x; i < N; i += 256) {
        const double x = s[o + i], y = s[SP + o + i], z = s[2 * SP + o + i];
        const double gx = GX[o + i], gy = GX[SP + o + i], uz = UZ[o + i], d = dg[i];
        const double xg = x * gx + y * gy;
        a0 += xg;
        a1 += d * z;
        a2 += z * (gx * gx + gy * gy);
        a3 += d * d * z;
        a4 += z * uz;
        a5 += d * xg;
    }
    const int t = threadIdx.x;
    red[0][t] = a0;
    red[1][t] = a1;
    red[2][t] = a2;
    red[3][t] = a3;
    red[4][t] = a4;
    red[5][t] = a5;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < 6; ++q) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t == 0) {
        const double E2 = 0.25 * red[0][0], D = red[1][0], Q3 = 0.25 * red[2][0], R = red[3][0], U = red[4][0],
                     V = 0.25 * red[5][0];
        const double v[9] = {E2, E2 * E2, E2 * D, Q3, R, D * D, U, V, D};
#pragma unroll
        for (int m = 0; m < 9; ++m) kahan_add(gmom[(2 * m) * Bp + k], gmom[(2 * m + 1) * Bp + k], v[m]);
    }
}

template <int PREC>
int build_ops_t(const Geometry& g, const double* G, const EnsembleBuffers& b, hipStream_t st) {
    typedef typename Prec<PREC>::G GT;
    typedef typename Prec<PREC>::S S;
    hipLaunchKernelGGL(decay_ops_kernel<PREC>, dim3(nblk(g.P * g.P, 256)), dim3(256), 0, st, G, g.N, g.P, g.kt,
                       static_cast<GT*>(b.AG), static_cast<GT*>(b.AGG), static_cast<S*>(b.dg));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <int PREC>
int observe_t(const Geometry& g, const EnsembleBuffers& b, int cur, hipStream_t st) {
    typedef typename Prec<PREC>::G GT;
    typedef typename Prec<PREC>::S S;
    int rc;
    // G [s^x, s^y]: the state part of the next step's operand
    GemmCall c{};
    c.kind = 2;
    c.stage = 1;
    c.A = b.AG;
    c.X = b.Xop;
    c.ldx = (2 + g.coh) * g.P;   // the state block leads every operand column
    c.K = g.P;
    c.Sout = b.GX;
    c.store_sign = 1.0;
    if ((rc = launch_gemm_call(g, c, st))) return rc;
    // (G o G) s^z over Bp / 2 column pairs
    hipLaunchKernelGGL(pack_z_kernel<PREC>, dim3(nblk(g.Bp * g.P, 256)), dim3(256), 0, st,
                       static_cast<const S*>(b.s[cur]), g.Bp, g.P, static_cast<GT*>(b.Zop));
    TWA_HIP_CHECK(hipGetLastError());
    Geometry gz = g;
    gz.Bp = g.Bp / 2;
    gz.C2 = g.Bp;
    GemmCall u{};
    u.kind = 2;
    u.stage = 1;
    u.A = b.AGG;
    u.X = b.Zop;
    u.ldx = g.P;
    u.K = g.P;
    u.Sout = b.UZ;
    u.store_sign = 1.0;
    if ((rc = launch_gemm_call(gz, u, st))) return rc;
    hipLaunchKernelGGL(decay_reduce_kernel<S>, dim3((unsigned)g.B), dim3(256), 0, st,
                       static_cast<const S*>(b.s[cur]), static_cast<const S*>(b.GX), static_cast<const S*>(b.UZ),
                       static_cast<const S*>(b.dg), g.N, g.P, g.Bp, b.gmom);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

}  // namespace

int decay_geometry_ok(const Geometry& g) {
    const TileCfg& tc = tile_cfg(g.cfg);
    if (g.Bp % tc.nt != 0) {
        set_error("correlated decay: trajectory padding must be a multiple of the column tile");
        return TWA_EINVAL;
    }
    return TWA_OK;
}

int launch_decay_ops(const Geometry& g, const double* G, const EnsembleBuffers& b, hipStream_t st) {
    switch (g.precision) {
        case TWA_PREC_FP64: return build_ops_t<TWA_PREC_FP64>(g, G, b, st);
        case TWA_PREC_FP32: return build_ops_t<TWA_PREC_FP32>(g, G, b, st);
        case TWA_PREC_BF16: return build_ops_t<TWA_PREC_BF16>(g, G, b, st);
        case TWA_PREC_FP16: return build_ops_t<TWA_PREC_FP16>(g, G, b, st);
    }
    set_error("unknown precision");
    return TWA_EINVAL;
}

int launch_decay_observe(const Geometry& g, const EnsembleBuffers& b, int cur, hipStream_t st) {
    switch (g.precision) {
        case TWA_PREC_FP64: return observe_t<TWA_PREC_FP64>(g, b, cur, st);
        case TWA_PREC_FP32: return observe_t<TWA_PREC_FP32>(g, b, cur, st);
        case TWA_PREC_BF16: return observe_t<TWA_PREC_BF16>(g, b, cur, st);
        case TWA_PREC_FP16: return observe_t<TWA_PREC_FP16>(g, b, cur, st);
    }
    set_error("unknown precision");
    return TWA_EINVAL;
}

}  // namespace twa
