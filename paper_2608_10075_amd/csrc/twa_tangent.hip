// twa_tangent_w: forward-mode (tangent-linear) pathwise derivatives of the
// steady-state observables with respect to the pump amplitude w of Eq. (2),
// at fixed Philox noise.
//
// One tangent copy ds = d s / d w runs beside the Heun steps of Eq. (S1).
// The pump enters a step only through the fields, and at fixed alpha W is
// linear and its PSD square root F square-root homogeneous in w, so with
// Y = A [s; zeta] (A = [-dt/2 W | -sqrt(dt) F]) and Q = -sqrt(dt) F zeta its
// noise part, dH/dw = Y/w - Q/(2w) at fixed state.  Per step:
//   predictor (kind PRIMAL_WITH_Q): Y1 and Q stored, D kept;
//   tangent predictor (kind TANGENT + source): dH1 = A_left ds + (Gamma dt/2)
//       sum(ds) + Y1/w - Q/(2w), dD1 = df/ds ds + df/dH dH1;
//   corrector (kind PRIMAL, its field Y2 stored);
//   tangent corrector (kind TANGENT + source with Y2);
// and every observed state adds the tangents of its moments (T2, T3, T4, Z,
// ZZ) to per-trajectory sums.  Work: 5 N x N x 2B contraction units per step
// against 3 for a plain step (the adjoint sweep needs 11 for (w, alpha)).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "twa_device.h"
#include "twa_internal.h"
#include "twa_run.h"

namespace twa {

namespace {

// tangents of the moments of the observed state, summed over the window in
// FP64 per trajectory: dacc[m][k], m over (T2, T3, T4, Z, ZZ)
template <typename S>
__global__ __launch_bounds__(256) void observe_tangent_kernel(int64_t B, int64_t Bp, int64_t nmt, const S* part,
                                                              const S* tpart, double* dacc) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B) return;
    S s3[3], t3[3];
    tile_sums<S, 3>(part, nmt, Bp, k, 0, s3);
    tile_sums<S, 3>(tpart, nmt, Bp, k, 0, t3);
    const double Sx = s3[0], Sy = s3[1], Sz = s3[2], dSx = t3[0], dSy = t3[1], dSz = t3[2];
    const double T2 = 0.25 * (Sx * Sx + Sy * Sy);
    const double dT2 = 0.5 * (Sx * dSx + Sy * dSy);
    dacc[0 * Bp + k] += dT2;
    dacc[1 * Bp + k] += dT2 * Sz + T2 * dSz;
    dacc[2 * Bp + k] += 2.0 * T2 * dT2;
    dacc[3 * Bp + k] += dSz;
    dacc[4 * Bp + k] += 2.0 * Sz * dSz;
}

template <typename S>
int launch_observe_tangent(const Geometry& g, const EnsembleBuffers& b, double* dacc, hipStream_t st) {
    hipLaunchKernelGGL(observe_tangent_kernel<S>, dim3((unsigned)((g.B + 255) / 256)), dim3(256), 0, st, g.B, g.Bp,
                       g.nmt, static_cast<const S*>(b.part[0]), static_cast<const S*>(b.tpart[0]), dacc);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

}  // namespace

int run_tangent_w(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                  twa_observables* out, double* grads) {
    if (!p || !p->pump || !out || !grads || n_traj < 1 || n_steps < 1 || !(dt > 0) || !std::isfinite(dt) ||
        !(p->gamma > 0) || !std::isfinite(p->gamma)) {
        set_error("twa_tangent_w: need params with a pump, n_traj >= 1, n_steps >= 1, dt > 0, gamma > 0, outputs");
        return TWA_EINVAL;
    }
    const twa_pump* pump = p->pump;
    if (!pump->W || pump->G || pump->Om || !std::isfinite(pump->w) || !(pump->w > 0) ||
        !std::isfinite(pump->alpha)) {
        set_error("twa_tangent_w: needs a pump of Eq. (2) from twa_build_pump with w > 0");
        return TWA_EINVAL;
    }
    if (p->integrator != TWA_INT_HEUN || p->n_lags > 0 || p->pump_path != TWA_PUMP_DENSE ||
        p->precision < TWA_PREC_FP64 || p->precision > TWA_PREC_BF16X3) {
        set_error("twa_tangent_w: Heun, dense pump, no lags, a known precision");
        return TWA_EINVAL;
    }
    const int64_t N = pump->N, B = n_traj;
    const int64_t burnin = p->burnin < 0 ? n_steps / 2 : p->burnin;
    if (burnin >= n_steps) {
        set_error("twa_tangent_w: the averaging window is empty");
        return TWA_EINVAL;
    }
    const int cfg = p->tile_config >= 0 ? p->tile_config : pick_tile_cfg(p->precision, N, B);
    if (cfg >= n_tile_cfgs() || (p->precision == TWA_PREC_FP64 && cfg > 3)) {
        set_error("twa_tangent_w: unknown tile configuration");
        return TWA_EINVAL;
    }
    Geometry g = make_geometry(p->precision, cfg, N, B);
    const int J = (int)std::min<int64_t>(32, B);
    const int64_t KP = g.P * operand_split(p->precision);   // K extent of one operand block (split: hi, lo, hi)
    const size_t se = (size_t)state_elt_bytes(p->precision);
    const size_t plane = (size_t)g.Bp * g.P * se;
    hipStream_t st = (hipStream_t)p->stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) {
            set_error("twa_tangent_w: hipStreamCreate failed (no usable GPU?)");
            return TWA_EHIP;
        }
        st = own;
    }
    EnsembleBuffers b;
    void* Q = nullptr;
    double* dacc = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = TWA_OK;
    int cur = 0;
    float ms = 0.f;
    std::vector<double> hmom, hd;
    std::vector<float> hdiag;
    const int nblk_fin = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (B * N + 255) / 256));
    StepConsts c;
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
    const double inv_w = 1.0 / pump->w;

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

    // the tangent starts at zero: the initial sampling does not depend on w
    TWA_TRY(alloc_buffers(g, true, 0, J, b, st));
    TWA_HTRY(hipMalloc(&Q, 2 * plane));
    TWA_HTRY(hipMalloc((void**)&dacc, (size_t)5 * g.Bp * sizeof(double)));
    TWA_HTRY(hipMemsetAsync(dacc, 0, (size_t)5 * g.Bp * sizeof(double), st));
    TWA_TRY(launch_build_A(g, pump->W, pump->F, dt, b.A, st));
    TWA_TRY(launch_init_state(g, b, c, nullptr, st));
    TWA_TRY(launch_reduce_state(g, b.s[0], b.part[0], st));
    TWA_HTRY(hipMemsetAsync(b.step, 0, sizeof(int64_t), st));
    TWA_HTRY(hipEventCreate(&e0));
    TWA_HTRY(hipEventCreate(&e1));
    TWA_HTRY(hipEventRecord(e0, st));
    for (int64_t n = 0; n < n_steps; ++n) {
        TWA_TRY(launch_noise(g, b, c, st));
        GemmCall p1;   // predictor, also storing its noise part Q
        p1.kind = KIND_PRIMAL_WITH_Q; p1.stage = 1; p1.A = b.A; p1.X = b.Xop; p1.ldx = 2 * KP;
        p1.K = 2 * KP; p1.c1 = c.c1; p1.c2 = c.c2; p1.s_cur = b.s[cur]; p1.dlt = b.dlt; p1.Y = b.Y;
        p1.Dop = b.Dop; p1.Sout = Q; p1.part_prim = b.part[0]; p1.part_out = b.part[1]; p1.g = b.g; p1.step = b.step;
        TWA_TRY(launch_gemm_call(g, p1, st));
        GemmCall t1;   // tangent predictor with the w-source
        t1.kind = 1; t1.stage = 1; t1.ncopy = 1; t1.A = b.A; t1.X = b.tXop; t1.ldx = KP;
        t1.K = KP; t1.c1 = c.c1; t1.c2 = c.c2; t1.s_cur = b.s[cur]; t1.Y = b.Y; t1.g = b.g;
        t1.part_prim = b.part[0]; t1.tpart_in = b.tpart[0]; t1.part_out = b.tpart[1]; t1.t_cur = b.ts[cur];
        t1.t_dlt = b.tdlt; t1.tY = b.tY; t1.tDop = b.tDop; t1.Qin = Q; t1.inv_w = inv_w;
        TWA_TRY(launch_gemm_call(g, t1, st));
        GemmCall p2;   // corrector, its field Y2 stored in place of Y1
        p2.kind = 0; p2.stage = 2; p2.A = b.A; p2.X = b.Dop; p2.ldx = KP; p2.K = KP;
        p2.c1 = c.c1; p2.c2 = c.c2; p2.s_cur = b.s[cur]; p2.s_next = b.s[1 - cur]; p2.dlt = b.dlt; p2.Y = b.Y;
        p2.store_y2 = 1; p2.part_prim = b.part[1]; p2.part_out = b.part[0]; p2.Xnext = b.Xop; p2.ldxn = 2 * KP;
        p2.g = b.g; p2.step = b.step;
        TWA_TRY(launch_gemm_call(g, p2, st));
        GemmCall t2;   // tangent corrector with the w-source at the corrector's field
        t2.kind = 1; t2.stage = 2; t2.ncopy = 1; t2.A = b.A; t2.X = b.tDop; t2.ldx = KP;
        t2.K = KP; t2.c1 = c.c1; t2.c2 = c.c2; t2.s_cur = b.s[cur]; t2.dlt = b.dlt; t2.Y = b.Y; t2.g = b.g;
        t2.part_prim = b.part[1]; t2.tpart_in = b.tpart[1]; t2.part_out = b.tpart[0]; t2.t_cur = b.ts[cur];
        t2.t_next = b.ts[1 - cur]; t2.t_dlt = b.tdlt; t2.tY = b.tY; t2.Xnext = b.tXop; t2.ldxn = KP; t2.Qin = Q;
        t2.inv_w = inv_w;
        TWA_TRY(launch_gemm_call(g, t2, st));
        if (n + 1 > burnin) {
            TWA_TRY(launch_observe(g, b, c, 1 - cur, false, st));
            if (p->precision == TWA_PREC_FP64) TWA_TRY(launch_observe_tangent<double>(g, b, dacc, st));
            else TWA_TRY(launch_observe_tangent<float>(g, b, dacc, st));
        }
        cur = 1 - cur;
    }
    TWA_HTRY(hipEventRecord(e1, st));
    TWA_TRY(launch_finish(g, b, cur, nblk_fin, st));
    hmom.resize((size_t)10 * g.Bp);
    hd.resize((size_t)5 * g.Bp);
    hdiag.resize((size_t)2 * nblk_fin);
    if (se == 8) {
        TWA_HTRY(hipMemcpyAsync(hmom.data(), b.mom, hmom.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    } else {
        std::vector<float> tmp(hmom.size());
        TWA_HTRY(hipMemcpyAsync(tmp.data(), b.mom, tmp.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        TWA_HTRY(hipStreamSynchronize(st));
        for (size_t i = 0; i < tmp.size(); ++i) hmom[i] = tmp[i];
    }
    TWA_HTRY(hipMemcpyAsync(hd.data(), dacc, hd.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    TWA_HTRY(hipMemcpyAsync(hdiag.data(), b.diag, hdiag.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    TWA_HTRY(hipStreamSynchronize(st));
    TWA_HTRY(hipEventElapsedTime(&ms, e0, e1));
    {
        const int64_t ns = n_steps - burnin;
        std::vector<double> traj((size_t)B * 5);
        bool nan = false;
        double m[5] = {0, 0, 0, 0, 0}, dm[5] = {0, 0, 0, 0, 0};
        for (int64_t k = 0; k < B; ++k)
            for (int q = 0; q < 5; ++q) {
                traj[(size_t)k * 5 + q] =
                    (hmom[(size_t)(2 * q) * g.Bp + k] - hmom[(size_t)(2 * q + 1) * g.Bp + k]) / (double)ns;
                dm[q] += hd[(size_t)q * g.Bp + k] / (double)ns;
            }
        std::memset(out, 0, sizeof(*out));
        finalize_moments(traj, B, out);
        for (int q = 0; q < 5; ++q) dm[q] /= (double)B;
        m[0] = out->T2; m[1] = out->T3; m[2] = out->T4; m[3] = out->Z; m[4] = out->ZZ;
        // chain rule on the ensemble moments; g2 by the quotient rule
        const double den = m[0] + 0.5 * m[3];
        const double num = m[2] + 2.0 * m[1] - m[3] / 3.0 + 0.5 * m[4] - (4.0 / 3.0) * m[0];
        const double dden = dm[0] + 0.5 * dm[3];
        const double dnum = dm[2] + 2.0 * dm[1] - dm[3] / 3.0 + 0.5 * dm[4] - (4.0 / 3.0) * dm[0];
        grads[0] = dden;
        grads[1] = dnum / (den * den) - 2.0 * (num / (den * den)) * dden / den;
        grads[2] = dm[3];
        double mx = 0;
        for (int i = 0; i < nblk_fin; ++i) {
            mx = std::max(mx, (double)hdiag[(size_t)i]);
            if (hdiag[(size_t)nblk_fin + i] != 0.f) nan = true;
        }
        for (int q = 0; q < 3; ++q)
            if (!std::isfinite(grads[q])) nan = true;
        out->n_samples = ns;
        out->max_norm_dev = mx;
        out->step_criterion = std::max(p->gamma * (double)N, pump->lam_max) * dt;
        out->nan_flag = nan ? 1 : 0;
        out->tile_config = cfg;
        out->kernel_ms = ms;
        out->gemm_flops = 20.0 * (double)N * (double)N * (double)B * (double)n_steps;
        out->linewidth = out->linewidth_sym = NAN;
        out->I_gen = out->g2_gen = out->I_gen_se = out->g2_gen_se = NAN;
        rc = run_status("twa_tangent_w", nan, mx, p->norm_tol);
    }
cleanup:
    if (rc != TWA_OK && rc != TWA_EUNSTABLE) hipStreamSynchronize(st);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(Q);
    hipFree(dacc);
    free_buffers(b);
    if (own) hipStreamDestroy(own);
#undef TWA_TRY
#undef TWA_HTRY
    return rc;
}

}  // namespace twa

extern "C" {

TWA_API int twa_tangent_w(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                          twa_observables* out, double* grads) {
    TWA_API_LOCK();
    return twa::run_tangent_w(p, n_traj, dt, n_steps, seed, out, grads);
}

}  // extern "C"
