// twa_run_batch: an uneven phase-diagram scan of many independent (N, w,
// alpha) points (each a full ensemble of Eq. (S1) trajectories) advanced in
// lockstep.  Every stage of every step is ONE grouped persistent launch over
// the tiles of all points (longest contraction first), the step sequence is
// captured in hipGraphs and replayed, and the tile configuration of the scan
// is chosen by measurement (cached on disk when a cache file is given).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "twa_device.h"
#include "twa_internal.h"
#include "twa_run.h"

namespace twa {

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// per-point description used by the grouped noise and observation kernels
struct PointDesc {
    int64_t N, B, P, Bp, nmt, burnin;
    uint32_t key0, key1, point;
    void* Xop;
    void* g;
    const void* part0;
    void* mom;
};

// noise of every point for the current step; block b belongs to the point p
// with bstart[p] <= b < bstart[p + 1]
template <int PREC>
__global__ void noise_grouped_kernel(const PointDesc* __restrict__ pd, const int* __restrict__ bstart, int np,
                                     const int64_t* step) {
    typedef typename Prec<PREC>::S S;
    typedef typename Prec<PREC>::G G;
    const int b = blockIdx.x;
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (bstart[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const PointDesc d = pd[lo];
    const int64_t nslot = (d.N + 1) / 2;
    const int64_t t = (int64_t)(b - bstart[lo]) * blockDim.x + threadIdx.x;
    if (t >= d.B * nslot) return;
    const int64_t k = t / nslot, m = t % nslot;
    const uint32_t n = (uint32_t)step[0];
    const U4 w = philox4x32_10(U4{(uint32_t)m, (uint32_t)k, n, TAG_PUMP | (d.point << 8)}, d.key0, d.key1);
    S z0, z1, z2, z3;
    box_muller(w.x, w.y, z0, z1);
    box_muller(w.z, w.w, z2, z3);
    const int64_t i = 2 * m;
    G* cx = static_cast<G*>(d.Xop) + opcol(k, 0) * 2 * d.P + d.P;
    G* cy = static_cast<G*>(d.Xop) + opcol(k, 1) * 2 * d.P + d.P;
    cx[i] = Prec<PREC>::to_g(z0);
    cy[i] = Prec<PREC>::to_g(z1);
    if (i + 1 < d.N) {
        cx[i + 1] = Prec<PREC>::to_g(z2);
        cy[i + 1] = Prec<PREC>::to_g(z3);
    }
    if (m == 0) {
        const U4 v = philox4x32_10(U4{0u, (uint32_t)k, n, TAG_COLLECTIVE | (d.point << 8)}, d.key0, d.key1);
        S g0, g1;
        box_muller(v.x, v.y, g0, g1);
        S* gg = static_cast<S*>(d.g);
        gg[k] = g0;
        gg[d.Bp + k] = g1;
    }
}

template <typename S>
__device__ __forceinline__ void kahan_add2(S* sum, S* comp, S v) {
    const S s = *sum, c = *comp;
    const S y = v - c;
    const S t = s + y;
    *comp = (t - s) - y;
    *sum = t;
}

// window moments of every point (the same Kahan sums as the single-run path)
template <typename S>
__global__ __launch_bounds__(256) void observe_grouped_kernel(const PointDesc* __restrict__ pd, const int64_t* step) {
    const PointDesc d = pd[blockIdx.x];
    const int64_t kst = step[0];
    if (kst <= d.burnin) return;
    const S* part = static_cast<const S*>(d.part0);
    S* mom = static_cast<S*>(d.mom);
    for (int64_t k = threadIdx.x; k < d.B; k += blockDim.x) {
        S sxyz[3];
        tile_sums<S, 3>(part, d.nmt, d.Bp, k, 0, sxyz);
        const S Sx = sxyz[0], Sy = sxyz[1], Sz = sxyz[2];
        const S T2 = S(0.25) * (Sx * Sx + Sy * Sy);
        const S v[5] = {T2, T2 * Sz, T2 * T2, Sz, Sz * Sz};
#pragma unroll
        for (int m = 0; m < 5; ++m) kahan_add2(mom + (2 * m) * d.Bp + k, mom + (2 * m + 1) * d.Bp + k, v[m]);
    }
}

struct Batch {
    std::vector<Geometry> gs;
    std::vector<EnsembleBuffers> bs;
    std::vector<StepConsts> cs;
    std::vector<twa_pump*> pumps;   // not owned
    PointDesc* d_pd = nullptr;
    int* d_bstart = nullptr;
    int nblocks_noise = 0;
    int64_t* step = nullptr;
    GroupedPlan plan;
    void release() {
        for (auto& b : bs) {
            b.step = nullptr;   // shared counter, freed once below
            free_buffers(b);
        }
        bs.clear();
        hipFree(d_pd);
        hipFree(d_bstart);
        hipFree(step);
        d_pd = nullptr;
        d_bstart = nullptr;
        step = nullptr;
        grouped_free(plan);
    }
};

int build_batch(const twa_point* pts, int np, const twa_batch_opts* o, const std::vector<twa_pump*>& pumps, int cfg,
                Batch& bt, hipStream_t st) {
    int rc;
    bt.pumps = pumps;
    bt.gs.resize((size_t)np);
    bt.bs.resize((size_t)np);
    bt.cs.resize((size_t)np);
    const int64_t burnin = o->burnin < 0 ? o->n_steps / 2 : o->burnin;
    if (hipMalloc(&bt.step, sizeof(int64_t)) != hipSuccess) {
        set_error("twa_run_batch: allocation failed");
        return TWA_ENOMEM;
    }
    std::vector<PointDesc> pd((size_t)np);
    std::vector<int> bstart((size_t)np + 1, 0);
    for (int p = 0; p < np; ++p) {
        Geometry& g = bt.gs[(size_t)p];
        g = make_geometry(o->precision, cfg, pts[p].N, o->n_traj);
        g.integrator = o->integrator;
        EnsembleBuffers& b = bt.bs[(size_t)p];
        if ((rc = alloc_buffers(g, false, 0, (int)std::min<int64_t>(32, o->n_traj), b))) return rc;
        hipFree(b.step);
        b.step = bt.step;   // one step counter for the lockstep scan
        StepConsts& c = bt.cs[(size_t)p];
        const double dt = pts[p].dt;
        c.c1 = 0.5 * o->gamma * dt;
        c.c2 = std::sqrt(o->gamma * dt);
        c.s0z = o->s0z;
        c.key0 = (uint32_t)(pts[p].seed & 0xffffffffu);
        c.key1 = (uint32_t)(pts[p].seed >> 32);
        c.point = p;
        c.burnin = burnin;
        c.lag_stride = 1;
        c.n_lags = 0;
        c.J = (int)std::min<int64_t>(32, o->n_traj);
        if ((rc = launch_build_A(g, pumps[(size_t)p]->W, pumps[(size_t)p]->F, dt, b.A, st))) return rc;
        if ((rc = launch_init_state(g, b, c, nullptr, st))) return rc;
        if ((rc = launch_reduce_state(g, b.s[0], b.part[0], st))) return rc;
        pd[(size_t)p] = PointDesc{g.N, g.B, g.P, g.Bp, g.nmt, burnin, c.key0, c.key1, (uint32_t)p,
                                  b.Xop, b.g, b.part[0], b.mom};
        bstart[(size_t)p + 1] = bstart[(size_t)p] + (int)nblk(g.B * ((g.N + 1) / 2), 256);
    }
    bt.nblocks_noise = bstart[(size_t)np];
    TWA_HIP_CHECK(hipMalloc(&bt.d_pd, pd.size() * sizeof(PointDesc)));
    TWA_HIP_CHECK(hipMemcpy(bt.d_pd, pd.data(), pd.size() * sizeof(PointDesc), hipMemcpyHostToDevice));
    TWA_HIP_CHECK(hipMalloc(&bt.d_bstart, bstart.size() * sizeof(int)));
    TWA_HIP_CHECK(hipMemcpy(bt.d_bstart, bstart.data(), bstart.size() * sizeof(int), hipMemcpyHostToDevice));
    TWA_HIP_CHECK(hipMemsetAsync(bt.step, 0, sizeof(int64_t), st));
    return grouped_prepare(bt.gs, bt.bs, bt.cs, bt.step, bt.plan);
}

int batch_step(Batch& bt, int cur, bool observe, hipStream_t st) {
    int rc;
    const int np = (int)bt.gs.size();
    switch (bt.gs[0].precision) {
        case TWA_PREC_FP32:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_FP32>, dim3((unsigned)bt.nblocks_noise), dim3(256), 0, st,
                               bt.d_pd, bt.d_bstart, np, (const int64_t*)bt.step);
            break;
        case TWA_PREC_BF16:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_BF16>, dim3((unsigned)bt.nblocks_noise), dim3(256), 0, st,
                               bt.d_pd, bt.d_bstart, np, (const int64_t*)bt.step);
            break;
        case TWA_PREC_FP16:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_FP16>, dim3((unsigned)bt.nblocks_noise), dim3(256), 0, st,
                               bt.d_pd, bt.d_bstart, np, (const int64_t*)bt.step);
            break;
        default:
            set_error("twa_run_batch: precision must be FP32, BF16 or FP16");
            return TWA_EINVAL;
    }
    TWA_HIP_CHECK(hipGetLastError());
    if ((rc = grouped_launch(bt.plan, 1, cur, st))) return rc;
    if ((rc = grouped_launch(bt.plan, 2, cur, st))) return rc;
    if (observe) {
        hipLaunchKernelGGL(observe_grouped_kernel<float>, dim3((unsigned)np), dim3(256), 0, st,
                           (const PointDesc*)bt.d_pd, (const int64_t*)bt.step);
        TWA_HIP_CHECK(hipGetLastError());
    }
    return TWA_OK;
}

// the current state buffer flips every step; the grouped arguments for the
// state in s[cur] must match it, and so must the observation's partial sums,
// which always live in part[0] (written by the corrector)
int run_steps(Batch& bt, int64_t n0, int64_t n1, int64_t burnin, int& cur, bool use_graph, int GS, hipStream_t st,
              std::map<int, hipGraphExec_t>& cache, std::vector<hipGraph_t>& graphs) {
    int rc;
    int64_t n = n0;
    while (n < n1) {
        const bool obs = n + 1 > burnin;
        int64_t run = 1;
        while (n + run < n1 && run < GS && ((n + run + 1 > burnin) == obs)) ++run;
        if (use_graph && run == GS) {
            const int key = (obs ? 2 : 0) + cur;
            auto it = cache.find(key);
            if (it == cache.end()) {
                hipGraph_t gr;
                TWA_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                int cc = cur, crc = TWA_OK;
                for (int s = 0; s < GS && crc == TWA_OK; ++s) {
                    crc = batch_step(bt, cc, obs, st);
                    cc = 1 - cc;
                }
                hipError_t ee = hipStreamEndCapture(st, &gr);
                if (crc) return crc;
                TWA_HIP_CHECK(ee);
                graphs.push_back(gr);
                hipGraphExec_t ex;
                TWA_HIP_CHECK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
                it = cache.emplace(key, ex).first;
            }
            TWA_HIP_CHECK(hipGraphLaunch(it->second, st));
            n += GS;
        } else {
            if ((rc = batch_step(bt, cur, obs, st))) return rc;
            cur = 1 - cur;
            n += 1;
        }
    }
    return TWA_OK;
}

std::string tune_key(const twa_point* pts, int np, const twa_batch_opts* o) {
    std::ostringstream s;
    s << "prec" << o->precision << ":int" << o->integrator << ":B" << o->n_traj << ":N";
    for (int p = 0; p < np; ++p) s << (p ? "," : "") << pts[p].N;
    return s.str();
}

int cached_cfg(const char* path, const std::string& key) {
    if (!path) return -1;
    std::ifstream f(path);
    std::string k;
    int c;
    while (f >> k >> c)
        if (k == key) return c;
    return -1;
}

void store_cfg(const char* path, const std::string& key, int cfg) {
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << cfg << "\n";
}

}  // namespace

// measures a few grouped steps for each candidate tile configuration
static int autotune(const twa_point* pts, int np, const twa_batch_opts* o, const std::vector<twa_pump*>& pumps,
                    hipStream_t st, int* best_cfg, double* best_ms) {
    const int cands[] = {2, 3, 1, 7};
    *best_cfg = -1;
    *best_ms = 1e300;
    for (int cfg : cands) {
        if (cfg == 7 && o->precision == TWA_PREC_FP64) continue;
        Batch bt;
        int rc = build_batch(pts, np, o, pumps, cfg, bt, st);
        if (rc == TWA_OK) {
            int cur = 0;
            rc = batch_step(bt, cur, false, st);   // warm-up
            cur = 1 - cur;
            hipEvent_t a, b;
            hipEventCreate(&a);
            hipEventCreate(&b);
            hipEventRecord(a, st);
            for (int s = 0; s < 4 && rc == TWA_OK; ++s) {
                rc = batch_step(bt, cur, false, st);
                cur = 1 - cur;
            }
            hipEventRecord(b, st);
            hipStreamSynchronize(st);
            float ms = 0.f;
            hipEventElapsedTime(&ms, a, b);
            hipEventDestroy(a);
            hipEventDestroy(b);
            if (rc == TWA_OK && ms < *best_ms) {
                *best_ms = ms;
                *best_cfg = cfg;
            }
        }
        bt.release();
        if (rc == TWA_ENOMEM) continue;
        if (rc != TWA_OK) return rc;
    }
    if (*best_cfg < 0) {
        set_error("twa_run_batch: no tile configuration fits");
        return TWA_ENOMEM;
    }
    return TWA_OK;
}

int run_batch(const twa_point* pts, int np, const twa_batch_opts* o, twa_observables* outs) {
    if (!pts || np < 1 || !o || !outs || o->n_traj < 1 || o->n_steps < 1 || !(o->gamma > 0)) {
        set_error("twa_run_batch: need points, options, outputs, n_traj >= 1, n_steps >= 1, gamma > 0");
        return TWA_EINVAL;
    }
    if (o->integrator != TWA_INT_HEUN && o->integrator != TWA_INT_SIB) {
        set_error("twa_run_batch: integrator must be TWA_INT_HEUN or TWA_INT_SIB");
        return TWA_EINVAL;
    }
    if (o->precision != TWA_PREC_FP32 && o->precision != TWA_PREC_BF16 && o->precision != TWA_PREC_FP16) {
        set_error("twa_run_batch: precision must be FP32, BF16 or FP16");
        return TWA_EINVAL;
    }
    for (int p = 0; p < np; ++p)
        if (pts[p].N < 1 || !(pts[p].dt > 0) || !std::isfinite(pts[p].w) || !std::isfinite(pts[p].alpha) ||
            pts[p].w < 0 || pts[p].alpha < 0) {
            set_error("twa_run_batch: point " + std::to_string(p) + " is invalid");
            return TWA_EINVAL;
        }
    const int64_t burnin = o->burnin < 0 ? o->n_steps / 2 : o->burnin;
    if (burnin >= o->n_steps) {
        set_error("twa_run_batch: the averaging window is empty");
        return TWA_EINVAL;
    }
    hipStream_t st = (hipStream_t)o->stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreate(&own) != hipSuccess) {
            set_error("twa_run_batch: hipStreamCreate failed (no usable GPU?)");
            return TWA_EHIP;
        }
        st = own;
    }
    std::vector<twa_pump*> pumps((size_t)np, nullptr);
    Batch bt;
    std::map<int, hipGraphExec_t> cache;
    std::vector<hipGraph_t> graphs;
    int rc = TWA_OK;
    int cfg = -1;
    double tune_ms = 0;
    int cur = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float loop_ms = 0.f;
    const std::string key = tune_key(pts, np, o);
    const int GS = o->steps_per_graph > 0 ? (o->steps_per_graph + 1) / 2 * 2 : 16;
    for (int p = 0; p < np && rc == TWA_OK; ++p) rc = twa_build_pump(pts[p].N, pts[p].w, pts[p].alpha, &pumps[(size_t)p]);
    if (rc) goto cleanup;
    cfg = cached_cfg(o->tune_cache, key);
    if (cfg < 0 || (cfg > 3 && cfg != 7) || (cfg == 7 && o->precision == TWA_PREC_FP64)) {
        if ((rc = autotune(pts, np, o, pumps, st, &cfg, &tune_ms))) goto cleanup;
        store_cfg(o->tune_cache, key, cfg);
    }
    if ((rc = build_batch(pts, np, o, pumps, cfg, bt, st))) goto cleanup;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipEventRecord(e0, st);
    if ((rc = run_steps(bt, 0, o->n_steps, burnin, cur, o->use_graph != 0, GS, st, cache, graphs))) goto cleanup;
    hipEventRecord(e1, st);
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("twa_run_batch: step kernels failed");
        rc = TWA_EHIP;
        goto cleanup;
    }
    hipEventElapsedTime(&loop_ms, e0, e1);
    for (int p = 0; p < np; ++p) {
        const Geometry& g = bt.gs[(size_t)p];
        const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (g.B * g.N + 255) / 256));
        if ((rc = launch_finish(g, bt.bs[(size_t)p], cur, nb, st))) goto cleanup;
        std::vector<float> mom((size_t)10 * g.Bp), diag((size_t)2 * nb);
        if (hipMemcpyAsync(mom.data(), bt.bs[(size_t)p].mom, mom.size() * sizeof(float), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipMemcpyAsync(diag.data(), bt.bs[(size_t)p].diag, diag.size() * sizeof(float), hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("twa_run_batch: copy-back failed");
            rc = TWA_EHIP;
            goto cleanup;
        }
        const int64_t ns = o->n_steps - burnin;
        std::vector<double> traj((size_t)g.B * 5);
        bool nan = false;
        for (int64_t k = 0; k < g.B; ++k)
            for (int m = 0; m < 5; ++m) {
                const double v =
                    ((double)mom[(size_t)(2 * m) * g.Bp + k] - (double)mom[(size_t)(2 * m + 1) * g.Bp + k]) / (double)ns;
                traj[(size_t)k * 5 + m] = v;
                if (!std::isfinite(v)) nan = true;
            }
        twa_observables& out = outs[p];
        std::memset(&out, 0, sizeof(out));
        finalize_moments(traj, g.B, &out);
        double mx = 0;
        for (int i = 0; i < nb; ++i) {
            mx = std::max(mx, (double)diag[(size_t)i]);
            if (diag[(size_t)nb + i] != 0.f) nan = true;
        }
        out.n_samples = ns;
        out.max_norm_dev = mx;
        out.step_criterion = std::max(o->gamma * (double)g.N, pumps[(size_t)p]->lam_max) * pts[p].dt;
        out.nan_flag = nan ? 1 : 0;
        out.tile_config = cfg;
        out.kernel_ms = loop_ms;   // the whole scan's step loop
        out.gemm_flops = 12.0 * (double)g.N * (double)g.N * (double)g.B * (double)o->n_steps;
        out.linewidth = NAN;
        out.I_gen = out.g2_gen = out.I_gen_se = out.g2_gen_se = NAN;
        out.linewidth_sym = NAN;
        if (nan) rc = TWA_EUNSTABLE;
    }
    if (rc == TWA_EUNSTABLE) set_error("twa_run_batch: non-finite values in some point");
cleanup:
    if (rc != TWA_OK && rc != TWA_EUNSTABLE) hipStreamSynchronize(st);
    for (auto& e : cache) hipGraphExecDestroy(e.second);
    for (auto& gr : graphs) hipGraphDestroy(gr);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    bt.release();
    for (auto* p : pumps) twa_pump_free(p);
    if (own) hipStreamDestroy(own);
    return rc;
}

}  // namespace twa

extern "C" {

TWA_API void twa_batch_opts_default(twa_batch_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_traj = 512;
    o->n_steps = 1000;
    o->burnin = -1;
    o->gamma = 1.0;
    o->s0z = 1.0;
    o->precision = TWA_PREC_FP32;
    o->use_graph = 1;
    o->steps_per_graph = 16;
    o->tune_cache = nullptr;
    o->stream = nullptr;
    o->integrator = TWA_INT_HEUN;
}

TWA_API int twa_run_batch(const twa_point* pts, int n_points, const twa_batch_opts* o, twa_observables* outs) {
    return twa::run_batch(pts, n_points, o, outs);
}

}  // extern "C"
