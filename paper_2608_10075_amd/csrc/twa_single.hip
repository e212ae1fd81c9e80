// twa_run: one ensemble of trajectories of Eq. (S1) on one device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "twa_internal.h"
#include "twa_run.h"

namespace twa {

int launch_step_kernels(const Geometry& g, EnsembleBuffers& b, const StepConsts& c, int cur, bool tan_active,
                        GemmTimers* tm, hipStream_t st) {
    int rc;
    if ((rc = launch_noise(g, b, c, st))) return rc;
    if (tm) tm->s1.begin(st);
    // the primal predictor increment is stored only when the response copies
    // of the step read it; otherwise the corrector recomputes it
    if ((rc = launch_gemm(g, b, c, 1, false, cur, false, tan_active, st))) return rc;
    if (tm) tm->s1.end(st);
    if (tan_active && (rc = launch_gemm(g, b, c, 1, true, cur, false, true, st))) return rc;
    if (tm) tm->s2.begin(st);
    if ((rc = launch_gemm(g, b, c, 2, false, cur, tan_active, tan_active, st))) return rc;
    if (tm) tm->s2.end(st);
    if (tan_active && (rc = launch_gemm(g, b, c, 2, true, cur, false, true, st))) return rc;
    return TWA_OK;
}

namespace {

struct StepKind {
    bool tan_active, seed_after, observe, tobs;
    int key() const { return (tan_active ? 1 : 0) | (seed_after ? 2 : 0) | (observe ? 4 : 0) | (tobs ? 8 : 0); }
};

struct Plan {
    int64_t burnin, L, stride, tan_end;
    StepKind kind(int64_t n) const {
        StepKind k;
        k.tan_active = L > 0 && n >= burnin && n < tan_end;
        k.seed_after = L > 0 && n + 1 == burnin;
        k.observe = (n + 1 > burnin) || k.seed_after;
        k.tobs = L > 0 && n + 1 >= burnin && n + 1 <= tan_end;
        return k;
    }
};

int one_step(const Geometry& g, EnsembleBuffers& b, const StepConsts& c, int& cur, const StepKind& k,
             bool decay, GemmTimers* tm, hipStream_t st) {
    int rc;
    if ((rc = launch_step_kernels(g, b, c, cur, k.tan_active, tm, st))) return rc;
    if (k.seed_after && (rc = launch_seed_tangents(g, b, 1 - cur, st))) return rc;
    if (k.observe && (rc = launch_observe(g, b, c, 1 - cur, k.tobs, st))) return rc;
    if (decay && k.observe && (rc = launch_decay_observe(g, b, 1 - cur, st))) return rc;
    cur = 1 - cur;
    return TWA_OK;
}

struct GraphCache {
    std::map<int, hipGraphExec_t> exec;
    std::vector<hipGraph_t> graphs;
    ~GraphCache() {
        for (auto& e : exec) hipGraphExecDestroy(e.second);
        for (auto& gr : graphs) hipGraphDestroy(gr);
    }
};

}  // namespace

int run_single(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
               twa_observables* out, const twa_outputs* outs) {
    const bool decay = p && p->pump && p->pump->G;
    if (!p || !p->pump || !out || n_traj < 1 || n_steps < 0 || !(dt > 0) || !std::isfinite(dt) ||
        (!decay && (!(p->gamma > 0) || !std::isfinite(p->gamma))) ||
        (p->integrator != TWA_INT_HEUN && p->integrator != TWA_INT_SIB)) {
        set_error("twa_run: need params with a pump, n_traj >= 1, n_steps >= 0, dt > 0, gamma > 0, "
                  "integrator TWA_INT_HEUN or TWA_INT_SIB");
        return TWA_EINVAL;
    }
    const bool toep = p->pump_path == TWA_PUMP_TOEPLITZ;
    if (p->pump_path != TWA_PUMP_DENSE && !toep) {
        set_error("twa_run: pump_path must be TWA_PUMP_DENSE or TWA_PUMP_TOEPLITZ");
        return TWA_EINVAL;
    }
    if (toep && (decay || !std::isfinite(p->pump->w) || !std::isfinite(p->pump->alpha) || p->n_lags > 0 ||
                 p->integrator != TWA_INT_HEUN ||
                 (p->precision != TWA_PREC_FP64 && p->precision != TWA_PREC_FP32) ||
                 p->pump->N > toeplitz_max_n(p->precision))) {
        set_error("twa_run: the Toeplitz path needs a pump from twa_build_pump, Heun, FP64 (N <= 8193) or FP32 "
                  "(N <= 16385) and no two-time lags");
        return TWA_EINVAL;
    }
    if (!toep && !p->pump->W) {
        set_error("twa_run: a handle from twa_build_pump_toeplitz runs only with pump_path = TWA_PUMP_TOEPLITZ");
        return TWA_EINVAL;
    }
    if (decay && p->n_lags > 0) {
        set_error("twa_run: the two-time correlation is not defined for correlated decay (n_lags must be 0)");
        return TWA_EINVAL;
    }
    if (p->integrator == TWA_INT_SIB && p->n_lags > 0) {
        set_error("twa_run: the two-time response copies are defined for the Heun integrator (n_lags must be 0)");
        return TWA_EINVAL;
    }
    if (p->precision < TWA_PREC_FP64 || p->precision > TWA_PREC_BF16X3) {
        set_error("twa_run: unknown precision");
        return TWA_EINVAL;
    }
    if (p->precision == TWA_PREC_BF16X3 && p->pump && p->pump->G) {
        set_error("twa_run: the split-BF16 precision runs without a decay matrix");
        return TWA_EINVAL;
    }
    const twa_pump* pump = p->pump;
    const int64_t N = pump->N, B = n_traj;
    const int64_t burnin = p->burnin < 0 ? n_steps / 2 : p->burnin;
    if (burnin > n_steps) {
        set_error("twa_run: burnin exceeds n_steps");
        return TWA_EINVAL;
    }
    const int64_t L = std::max<int64_t>(0, p->n_lags);
    int64_t stride = 1;
    if (L > 0) {
        stride = p->lag_stride > 0 ? p->lag_stride : std::max<int64_t>(1, (n_steps - burnin) / L);
        if ((L - 1) * stride > n_steps - burnin) {
            set_error("twa_run: (n_lags - 1) * lag_stride exceeds the window");
            return TWA_EINVAL;
        }
    }
    int cfg = toep ? 0 : p->tile_config >= 0 ? p->tile_config : pick_tile_cfg(p->precision, N, B);
    if (cfg >= n_tile_cfgs() || (p->precision == TWA_PREC_FP64 && cfg > 3)) {
        set_error("twa_run: unknown tile configuration");
        return TWA_EINVAL;
    }
    Geometry g = make_geometry(p->precision, cfg, N, B);
    g.integrator = p->integrator;
    g.coh = pump->Om ? 1 : 0;
    if (decay) {
        // the packed s^z contraction covers Bp / 2 column pairs
        g.Bp = round_up(B, tile_cfg(cfg).nt);
        g.C2 = 2 * g.Bp;
    }
    const bool fused = p->tile_config < 0 && !decay && !toep && small_path_applies(p->precision, N, L);
    const int J = (int)std::min<int64_t>(32, B);
    const bool tangents = L > 0;

    hipStream_t st = (hipStream_t)p->stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) {
            set_error("twa_run: hipStreamCreate failed (no usable GPU?)");
            return TWA_EHIP;
        }
        st = own;
    }
    EnsembleBuffers b;
    double* init_dev = nullptr;
    double* export_dev = nullptr;
    void *toep_tw = nullptr, *toep_spec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GemmTimers* tm = nullptr;
    GraphCache gc;
    int rc = TWA_OK;
    std::vector<double> hmom, hlag, hgen;
    std::vector<float> hdiag;
    const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (B * N + 255) / 256));

    StepConsts c;
    // a decay matrix replaces the collective terms (it sits in the operand)
    c.c1 = decay ? 0.0 : 0.5 * p->gamma * dt;
    c.c2 = decay ? 0.0 : std::sqrt(p->gamma * dt);
    c.s0z = p->s0z;
    c.key0 = (uint32_t)(seed & 0xffffffffu);
    c.key1 = (uint32_t)(seed >> 32);
    c.point = p->point;
    c.burnin = burnin;
    c.lag_stride = stride;
    c.n_lags = L;
    c.J = J;
    Plan plan{burnin, L, stride, burnin + (L > 0 ? (L - 1) * stride : 0)};
    const bool use_graph = p->use_graph && !p->timing;
    const int GS = 16;   // steps per captured graph (even: the state ping-pong returns to its parity)
    int cur = 0;
    int64_t n = 0;
    float loop_ms = 0.f;

#define TWA_TRY(expr)                 \
    do {                              \
        if ((rc = (expr)) != TWA_OK) goto cleanup; \
    } while (0)
#define TWA_HTRY(expr)                                                   \
    do {                                                                 \
        hipError_t _e = (expr);                                          \
        if (_e != hipSuccess) {                                          \
            set_error(std::string(#expr) + ": " + hipGetErrorString(_e)); \
            rc = TWA_EHIP;                                               \
            goto cleanup;                                                \
        }                                                                \
    } while (0)

    TWA_TRY(alloc_buffers(g, tangents, L, J, b, st));
    if (toep)
        TWA_TRY(toeplitz_tables(g, pump->w, pump->alpha, dt, &toep_tw, &toep_spec, st));
    else if (g.coh)
        TWA_TRY(launch_build_A_coh(g, pump->W, pump->F, pump->Om, dt, b.A, b.A2, st));
    else
        TWA_TRY(launch_build_A(g, pump->W, pump->F, dt, b.A, st));
    if (decay) {
        TWA_TRY(decay_geometry_ok(g));
        TWA_TRY(alloc_decay_buffers(g, b, st));
        TWA_TRY(launch_decay_ops(g, pump->G, b, st));
    }
    if (p->init_state) {
        TWA_HTRY(hipMalloc(&init_dev, (size_t)3 * B * N * sizeof(double)));
        TWA_HTRY(hipMemcpyAsync(init_dev, p->init_state, (size_t)3 * B * N * sizeof(double), hipMemcpyHostToDevice, st));
    }
    TWA_TRY(launch_init_state(g, b, c, init_dev, st));
    TWA_TRY(launch_reduce_state(g, b.s[0], b.part[0], st));
    TWA_HTRY(hipMemsetAsync(b.step, 0, sizeof(int64_t), st));
    if (L > 0 && burnin == 0) {
        TWA_TRY(launch_seed_tangents(g, b, cur, st));
        TWA_TRY(launch_observe(g, b, c, cur, true, st));
    }
    if (p->timing) {
        tm = new GemmTimers();
        TWA_TRY(tm->s1.init());
        TWA_TRY(tm->s2.init());
    }
    TWA_HTRY(hipEventCreate(&e0));
    TWA_HTRY(hipEventCreate(&e1));
    TWA_HTRY(hipEventRecord(e0, st));
    if (fused) {
        // one launch integrates every step (short chains are bound by per-step latency)
        cur = (int)(n_steps & 1);
        TWA_TRY(launch_small_run(g, b, c, pump, dt, n_steps, cur, st));
        n = n_steps;
    }
    if (toep) {
        // one workgroup per trajectory, state updated in place
        TWA_TRY(launch_toeplitz_run(g, b, c, toep_tw, toep_spec, n_steps, cur, st));
        n = n_steps;
    }
    while (n < n_steps) {
        const StepKind k = plan.kind(n);
        int64_t run = 1;
        while (n + run < n_steps && run < GS && plan.kind(n + run).key() == k.key()) ++run;
        if (use_graph && run == GS && !k.seed_after) {
            const int key = k.key() * 2 + cur;
            auto it = gc.exec.find(key);
            if (it == gc.exec.end()) {
                hipGraph_t gr;
                TWA_HTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                int cc = cur;
                int crc = TWA_OK;
                for (int s = 0; s < GS && crc == TWA_OK; ++s) crc = one_step(g, b, c, cc, k, decay, nullptr, st);
                hipError_t ee = hipStreamEndCapture(st, &gr);
                if (crc != TWA_OK) {
                    rc = crc;
                    goto cleanup;
                }
                TWA_HTRY(ee);
                gc.graphs.push_back(gr);
                hipGraphExec_t ex;
                TWA_HTRY(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
                it = gc.exec.emplace(key, ex).first;
            }
            TWA_HTRY(hipGraphLaunch(it->second, st));
            n += GS;   // GS even: cur unchanged
        } else {
            TWA_TRY(one_step(g, b, c, cur, k, decay, tm, st));
            n += 1;
        }
    }
    TWA_HTRY(hipEventRecord(e1, st));
    TWA_TRY(launch_finish(g, b, cur, nblk, st));
    hmom.resize((size_t)10 * g.Bp);
    hdiag.resize((size_t)2 * nblk);
    if (g.precision == TWA_PREC_FP64) {
        TWA_HTRY(hipMemcpyAsync(hmom.data(), b.mom, hmom.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    } else {
        std::vector<float> tmp(hmom.size());
        TWA_HTRY(hipMemcpyAsync(tmp.data(), b.mom, tmp.size() * sizeof(float), hipMemcpyDeviceToHost, st));
        TWA_HTRY(hipStreamSynchronize(st));
        for (size_t i = 0; i < tmp.size(); ++i) hmom[i] = tmp[i];
    }
    TWA_HTRY(hipMemcpyAsync(hdiag.data(), b.diag, hdiag.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    if (decay) {
        hgen.resize((size_t)18 * g.Bp);
        TWA_HTRY(hipMemcpyAsync(hgen.data(), b.gmom, hgen.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    if (L > 0) {
        hlag.resize((size_t)L * J * 6);
        TWA_HTRY(hipMemcpyAsync(hlag.data(), b.lag, hlag.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    if (outs && outs->final_state) {
        TWA_HTRY(hipMalloc(&export_dev, (size_t)3 * B * N * sizeof(double)));
        TWA_TRY(launch_export_state(g, b.s[cur], export_dev, st));
        TWA_HTRY(hipMemcpyAsync(outs->final_state, export_dev, (size_t)3 * B * N * sizeof(double),
                                hipMemcpyDeviceToHost, st));
    }
    TWA_HTRY(hipStreamSynchronize(st));
    TWA_HTRY(hipEventElapsedTime(&loop_ms, e0, e1));
    {
        std::memset(out, 0, sizeof(*out));
        const int64_t ns = n_steps - burnin;
        std::vector<double> traj((size_t)B * 5);
        bool nan = false;
        for (int64_t k = 0; k < B; ++k)
            for (int m = 0; m < 5; ++m) {
                const double s = hmom[(size_t)(2 * m) * g.Bp + k], cmp = hmom[(size_t)(2 * m + 1) * g.Bp + k];
                const double v = ns > 0 ? (s - cmp) / (double)ns : NAN;
                traj[(size_t)k * 5 + m] = v;
                if (ns > 0 && !std::isfinite(v)) nan = true;
            }
        finalize_moments(traj, B, out);
        double mx = 0;
        for (int i = 0; i < nblk; ++i) {
            mx = std::max(mx, (double)hdiag[(size_t)i]);
            if (hdiag[(size_t)nblk + i] != 0.f) nan = true;
        }
        out->n_samples = ns;
        out->n_lags = L;
        out->lag_stride = stride;
        out->max_norm_dev = mx;
        out->step_criterion = (decay ? pump->lam_max : std::max(p->gamma * (double)N, pump->lam_max)) * dt;
        out->nan_flag = nan ? 1 : 0;
        out->tile_config = fused ? TWA_TILE_FUSED : toep ? TWA_TILE_TOEPLITZ : cfg;
        out->kernel_ms = loop_ms;
        if (tm) {
            tm->s1.harvest(st);
            tm->s2.harvest(st);
            out->stage1_ms = tm->s1.total_ms;
            out->stage1_launches = tm->s1.count;
            out->stage2_ms = tm->s2.total_ms;
            out->stage2_launches = tm->s2.count;
        }
        // algorithmic contraction flops: stage 1 2*N*(2N)*(2B), stage 2 2*N*N*(2B);
        // response copies: 2 copies x 2*N*N*(2B) per stage
        const double nb = (double)N * (double)N * (double)B;
        const double tan_steps = L > 0 ? (double)((L - 1) * stride) : 0.0;
        // correlated decay: G [s^x, s^y] and (G o G) s^z per observed state
        out->gemm_flops = toep ? 0.0
                               : (double)n_steps * 12.0 * nb + tan_steps * 16.0 * nb +
                                     (decay ? (double)ns * 6.0 * nb : 0.0);
        out->I_gen = out->g2_gen = out->I_gen_se = out->g2_gen_se = NAN;
        if (decay) {
            std::vector<double> tg((size_t)B * 9);
            for (int64_t k = 0; k < B; ++k)
                for (int m = 0; m < 9; ++m) {
                    const double s = hgen[(size_t)(2 * m) * g.Bp + k], cmp = hgen[(size_t)(2 * m + 1) * g.Bp + k];
                    const double v = ns > 0 ? (s - cmp) / (double)ns : NAN;
                    tg[(size_t)k * 9 + m] = v;
                    if (ns > 0 && !std::isfinite(v)) nan = true;
                }
            finalize_decay(tg, B, out);
            if (outs && outs->traj_gen) std::memcpy(outs->traj_gen, tg.data(), tg.size() * sizeof(double));
            out->nan_flag = nan ? 1 : 0;
        }
        out->linewidth = NAN;
        out->linewidth_sym = NAN;
        if (L > 0) finalize_lags(hlag, L, J, B, stride, dt, p->kappa, out, outs);
        if (outs && outs->traj_moments) std::memcpy(outs->traj_moments, traj.data(), traj.size() * sizeof(double));
        if (outs && outs->n_blocks) *outs->n_blocks = J;
        rc = run_status("twa_run", nan, mx, p->norm_tol);
    }
cleanup:
    if (rc != TWA_OK && rc != TWA_EUNSTABLE) hipStreamSynchronize(st);
    delete tm;
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(init_dev);
    hipFree(export_dev);
    hipFree(toep_tw);
    hipFree(toep_spec);
    free_buffers(b);
    if (own) hipStreamDestroy(own);
#undef TWA_TRY
#undef TWA_HTRY
    return rc;
}

}  // namespace twa
