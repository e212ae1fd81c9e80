// twa_run_batch: an uneven phase-diagram scan of many independent (N, w,
// alpha) points (each a full ensemble of Eq. (S1) trajectories).
//
// The points are split into buckets by N.  A bucket's points share a tile
// configuration (chosen per bucket by measurement, cached on disk when a cache
// file is given) and advance in lockstep: every stage of every step is ONE
// grouped persistent launch over the tiles of all the bucket's points,
// longest contraction first.  Each bucket has its own step counter and runs on
// its own stream branch; the steps of all buckets are captured together in
// hipGraphs (fork/join over the branches) and replayed, so a small-N bucket's
// launches fill the device while the large-N bucket's tail runs.
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
    int64_t N, B, P, Bp, nmt, burnin, L, stride;
    uint32_t key0, key1, point;
    int32_t pad_;
    void* Xop;
    void* g;
    const void* part0;
    void* mom;
    const void* tpart0;   // partial sums of the response copies (two-time)
    void* sm0;
    double* lag;
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
    // operand column: [s ; zeta], each block P long, or in the split form
    // (hi, lo, hi) blocks of P each for s and then for zeta
    constexpr int SPL = Prec<PREC>::SPLIT;
    G* cx = static_cast<G*>(d.Xop) + opcol(k, 0) * 2 * d.P * SPL + d.P * SPL;
    G* cy = static_cast<G*>(d.Xop) + opcol(k, 1) * 2 * d.P * SPL + d.P * SPL;
    put_op<PREC>(cx + i, d.P, z0);
    put_op<PREC>(cy + i, d.P, z1);
    if (i + 1 < d.N) {
        put_op<PREC>(cx + i + 1, d.P, z2);
        put_op<PREC>(cy + i + 1, d.P, z3);
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

// observation after a step, one workgroup per (point, jackknife block j):
// the window moments (Kahan time sums per trajectory, as in the single-run
// path), the two-time origin and the lag sums of block j
template <typename S>
__global__ __launch_bounds__(256) void observe_grouped_kernel(const PointDesc* __restrict__ pd, int J,
                                                              const int64_t* step, int tangents) {
    __shared__ double red[6][256];
    const int p = blockIdx.x / J, j = blockIdx.x % J;
    const PointDesc d = pd[p];
    const int64_t kst = step[0];
    const int64_t B = d.B, Bp = d.Bp, nmt = d.nmt, L = d.L;
    const int64_t klo = ((int64_t)j * B + J - 1) / J, khi = ((int64_t)(j + 1) * B + J - 1) / J;
    const bool in_window = kst > d.burnin;
    const bool origin = L > 0 && kst == d.burnin;
    int64_t l = -1;
    if (L > 0 && kst >= d.burnin && (kst - d.burnin) % d.stride == 0 && (kst - d.burnin) / d.stride < L)
        l = (kst - d.burnin) / d.stride;
    const S* part = static_cast<const S*>(d.part0);
    const S* tpart = static_cast<const S*>(d.tpart0);
    S* mom = static_cast<S*>(d.mom);
    S* sm0 = static_cast<S*>(d.sm0);
    double acc6[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = klo + threadIdx.x; k < khi; k += blockDim.x) {
        S sxyz[3];
        tile_sums<S, 3>(part, nmt, Bp, k, 0, sxyz);
        const S Sx = sxyz[0], Sy = sxyz[1], Sz = sxyz[2];
        if (in_window) {
            const S T2 = S(0.25) * (Sx * Sx + Sy * Sy);
            const S v[5] = {T2, T2 * Sz, T2 * T2, Sz, Sz * Sz};
#pragma unroll
            for (int m = 0; m < 5; ++m) kahan_add2(mom + (2 * m) * Bp + k, mom + (2 * m + 1) * Bp + k, v[m]);
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
                    tile_sums<S, 2>(tpart + cp * 3 * nmt * Bp, nmt, Bp, k, 0, txy);
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
    if (threadIdx.x < 6) d.lag[(l * J + j) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// the kind of a step of the shared plan (same for every point: all points
// share n_steps, the window and the lags)
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

// the points of one tile configuration, advanced in grouped launches
struct Bucket {
    int cfg = 0;
    std::vector<int> idx;            // positions in the caller's point list
    std::vector<Geometry> gs;
    std::vector<EnsembleBuffers> bs;
    std::vector<StepConsts> cs;
    PointDesc* d_pd = nullptr;
    int* d_bstart = nullptr;
    int nblocks_noise = 0;
    int J = 1;
    int64_t* step = nullptr;
    GroupedPlan plan;
    hipStream_t stream = nullptr;    // the branch this bucket runs on (not owned)
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

struct BatchSpec {
    const twa_point* pts;
    const twa_batch_opts* o;
    const std::vector<twa_pump*>* pumps;
    int64_t burnin, L, stride;
};

int launch_observe_grouped(Bucket& bk, bool tobs, hipStream_t st) {
    const int np = (int)bk.gs.size();
    if (bk.gs[0].precision == TWA_PREC_FP64)
        hipLaunchKernelGGL(observe_grouped_kernel<double>, dim3((unsigned)(np * bk.J)), dim3(256), 0, st,
                           (const PointDesc*)bk.d_pd, bk.J, (const int64_t*)bk.step, tobs ? 1 : 0);
    else
        hipLaunchKernelGGL(observe_grouped_kernel<float>, dim3((unsigned)(np * bk.J)), dim3(256), 0, st,
                           (const PointDesc*)bk.d_pd, bk.J, (const int64_t*)bk.step, tobs ? 1 : 0);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

int build_bucket(const BatchSpec& sp, const std::vector<int>& idx, int cfg, Bucket& bk, hipStream_t st) {
    int rc;
    const twa_batch_opts* o = sp.o;
    const int np = (int)idx.size();
    bk.cfg = cfg;
    bk.idx = idx;
    bk.gs.resize((size_t)np);
    bk.bs.resize((size_t)np);
    bk.cs.resize((size_t)np);
    bk.J = (int)std::min<int64_t>(32, o->n_traj);
    const bool tangents = sp.L > 0;
    if (hipMalloc(&bk.step, sizeof(int64_t)) != hipSuccess) {
        set_error("twa_run_batch: allocation failed");
        return TWA_ENOMEM;
    }
    std::vector<PointDesc> pd((size_t)np);
    std::vector<int> bstart((size_t)np + 1, 0);
    for (int q = 0; q < np; ++q) {
        const int p = idx[(size_t)q];
        const twa_point& pt = sp.pts[p];
        Geometry& g = bk.gs[(size_t)q];
        g = make_geometry(o->precision, cfg, pt.N, o->n_traj);
        g.integrator = o->integrator;
        EnsembleBuffers& b = bk.bs[(size_t)q];
        if ((rc = alloc_buffers(g, tangents, sp.L, bk.J, b, st))) return rc;
        hipFree(b.step);
        b.step = bk.step;   // one step counter for the bucket
        StepConsts& c = bk.cs[(size_t)q];
        c.c1 = 0.5 * o->gamma * pt.dt;
        c.c2 = std::sqrt(o->gamma * pt.dt);
        c.s0z = o->s0z;
        c.key0 = (uint32_t)(pt.seed & 0xffffffffu);
        c.key1 = (uint32_t)(pt.seed >> 32);
        c.point = p;
        c.burnin = sp.burnin;
        c.lag_stride = sp.stride;
        c.n_lags = sp.L;
        c.J = bk.J;
        const twa_pump* pump = (*sp.pumps)[(size_t)p];
        if ((rc = launch_build_A(g, pump->W, pump->F, pt.dt, b.A, st))) return rc;
        if ((rc = launch_init_state(g, b, c, nullptr, st))) return rc;
        if ((rc = launch_reduce_state(g, b.s[0], b.part[0], st))) return rc;
        PointDesc& d = pd[(size_t)q];
        d = PointDesc{};
        d.N = g.N;
        d.B = g.B;
        d.P = g.P;
        d.Bp = g.Bp;
        d.nmt = g.nmt;
        d.burnin = sp.burnin;
        d.L = sp.L;
        d.stride = sp.stride;
        d.key0 = c.key0;
        d.key1 = c.key1;
        d.point = (uint32_t)p;
        d.Xop = b.Xop;
        d.g = b.g;
        d.part0 = b.part[0];
        d.mom = b.mom;
        d.tpart0 = b.tpart[0];
        d.sm0 = b.sm0;
        d.lag = b.lag;
        bstart[(size_t)q + 1] = bstart[(size_t)q] + (int)nblk(g.B * ((g.N + 1) / 2), 256);
    }
    bk.nblocks_noise = bstart[(size_t)np];
    TWA_HIP_CHECK(hipMalloc(&bk.d_pd, pd.size() * sizeof(PointDesc)));
    TWA_HIP_CHECK(hipMemcpyAsync(bk.d_pd, pd.data(), pd.size() * sizeof(PointDesc), hipMemcpyHostToDevice, st));
    TWA_HIP_CHECK(hipMalloc(&bk.d_bstart, bstart.size() * sizeof(int)));
    TWA_HIP_CHECK(hipMemcpyAsync(bk.d_bstart, bstart.data(), bstart.size() * sizeof(int), hipMemcpyHostToDevice,
                                 st));
    TWA_HIP_CHECK(hipStreamSynchronize(st));   // the host arrays end with this function
    TWA_HIP_CHECK(hipMemsetAsync(bk.step, 0, sizeof(int64_t), st));
    if ((rc = grouped_prepare(bk.gs, bk.bs, bk.cs, bk.step, tangents, bk.plan, st))) return rc;
    if (sp.L > 0 && sp.burnin == 0) {
        // the origin is the initial state: seed the response copies and observe it
        for (int q = 0; q < np; ++q)
            if ((rc = launch_seed_tangents(bk.gs[(size_t)q], bk.bs[(size_t)q], 0, st))) return rc;
        if ((rc = launch_observe_grouped(bk, true, st))) return rc;
    }
    return TWA_OK;
}

// one step of one bucket (the step counter on the device advances in the
// corrector launch), on stream st
int bucket_step(Bucket& bk, int cur, const StepKind& k, hipStream_t st) {
    int rc;
    const int np = (int)bk.gs.size();
    const unsigned nb = (unsigned)bk.nblocks_noise;
    switch (bk.gs[0].precision) {
        case TWA_PREC_FP64:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_FP64>, dim3(nb), dim3(256), 0, st, bk.d_pd, bk.d_bstart,
                               np, (const int64_t*)bk.step);
            break;
        case TWA_PREC_FP32:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_FP32>, dim3(nb), dim3(256), 0, st, bk.d_pd, bk.d_bstart,
                               np, (const int64_t*)bk.step);
            break;
        case TWA_PREC_BF16:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_BF16>, dim3(nb), dim3(256), 0, st, bk.d_pd, bk.d_bstart,
                               np, (const int64_t*)bk.step);
            break;
        case TWA_PREC_FP16:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_FP16>, dim3(nb), dim3(256), 0, st, bk.d_pd, bk.d_bstart,
                               np, (const int64_t*)bk.step);
            break;
        case TWA_PREC_BF16X3:
            hipLaunchKernelGGL(noise_grouped_kernel<TWA_PREC_BF16X3>, dim3(nb), dim3(256), 0, st, bk.d_pd,
                               bk.d_bstart, np, (const int64_t*)bk.step);
            break;
        default:
            set_error("twa_run_batch: precision must be FP64, FP32, BF16, FP16 or split BF16");
            return TWA_EINVAL;
    }
    TWA_HIP_CHECK(hipGetLastError());
    const int pv = k.tan_active ? GV_PRIMAL_TAN : GV_PRIMAL;
    if ((rc = grouped_launch(bk.plan, 1, cur, pv, st))) return rc;
    if (k.tan_active && (rc = grouped_launch(bk.plan, 1, cur, GV_TANGENT, st))) return rc;
    if ((rc = grouped_launch(bk.plan, 2, cur, pv, st))) return rc;
    if (k.tan_active && (rc = grouped_launch(bk.plan, 2, cur, GV_TANGENT, st))) return rc;
    if (k.seed_after)
        for (int q = 0; q < np; ++q)
            if ((rc = launch_seed_tangents(bk.gs[(size_t)q], bk.bs[(size_t)q], 1 - cur, st))) return rc;
    if (k.observe && (rc = launch_observe_grouped(bk, k.tobs, st))) return rc;
    return TWA_OK;
}

// `run` consecutive steps of the same kind of every bucket, each bucket on its
// own branch: fork from st, the buckets' launches on their streams, join
// back into st (inside a capture the branches become parallel graph paths)
int buckets_steps(std::vector<Bucket>& bks, int cur, const StepKind& k, int run, hipStream_t st,
                  std::vector<hipEvent_t>& ev) {
    int rc;
    if (bks.size() == 1) {
        int cc = cur;
        for (int s = 0; s < run; ++s) {
            if ((rc = bucket_step(bks[0], cc, k, st))) return rc;
            cc = 1 - cc;
        }
        return TWA_OK;
    }
    TWA_HIP_CHECK(hipEventRecord(ev[0], st));
    for (size_t b = 0; b < bks.size(); ++b) {
        TWA_HIP_CHECK(hipStreamWaitEvent(bks[b].stream, ev[0], 0));
        int cc = cur;
        for (int s = 0; s < run; ++s) {
            if ((rc = bucket_step(bks[b], cc, k, bks[b].stream))) return rc;
            cc = 1 - cc;
        }
        TWA_HIP_CHECK(hipEventRecord(ev[1 + b], bks[b].stream));
        TWA_HIP_CHECK(hipStreamWaitEvent(st, ev[1 + b], 0));
    }
    return TWA_OK;
}

struct GraphSet {
    std::map<int, hipGraphExec_t> exec;
    std::vector<hipGraph_t> graphs;
    ~GraphSet() {
        for (auto& e : exec) hipGraphExecDestroy(e.second);
        for (auto& g : graphs) hipGraphDestroy(g);
    }
};

// steps n0 .. n1 - 1 of every bucket; runs of GS steps of one kind are
// replayed from captured graphs
int run_steps(std::vector<Bucket>& bks, const Plan& plan, int64_t n0, int64_t n1, int& cur, bool use_graph, int GS,
              int64_t progress, hipStream_t st, std::vector<hipEvent_t>& ev, GraphSet& gset) {
    int rc;
    int64_t n = n0;
    int64_t next_report = progress > 0 ? (n0 / progress + 1) * progress : INT64_MAX;
    while (n < n1) {
        const StepKind k = plan.kind(n);
        int64_t run = 1;
        while (n + run < n1 && run < GS && plan.kind(n + run).key() == k.key()) ++run;
        if (use_graph && run == GS && !k.seed_after) {
            const int key = k.key() * 2 + cur;
            auto it = gset.exec.find(key);
            if (it == gset.exec.end()) {
                hipGraph_t gr;
                TWA_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                const int crc = buckets_steps(bks, cur, k, GS, st, ev);
                hipError_t ee = hipStreamEndCapture(st, &gr);
                if (crc) return crc;
                TWA_HIP_CHECK(ee);
                gset.graphs.push_back(gr);
                hipGraphExec_t ex;
                TWA_HIP_CHECK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
                it = gset.exec.emplace(key, ex).first;
            }
            TWA_HIP_CHECK(hipGraphLaunch(it->second, st));
            n += GS;   // GS even: cur unchanged
        } else {
            if ((rc = buckets_steps(bks, cur, k, 1, st, ev))) return rc;
            cur = 1 - cur;
            n += 1;
        }
        if (n >= next_report) {
            TWA_HIP_CHECK(hipStreamSynchronize(st));
            std::fprintf(stderr, "[twa_run_batch] step %lld / %lld\n", (long long)n, (long long)n1);
            std::fflush(stderr);
            while (next_report <= n) next_report += progress;
        }
    }
    return TWA_OK;
}

// ---------------------------------------------------------------------------
// autotuning per N bucket
int bucket_of(int64_t N) { return N <= 128 ? 0 : N <= 1024 ? 1 : 2; }

std::vector<int> bucket_candidates(int bucket, int precision) {
    std::vector<int> c;
    if (bucket == 0) c = {0, 1};
    else if (bucket == 1) c = {1, 2, 3, 7};
    else c = {2, 3, 7};
    if (precision == TWA_PREC_FP64) c.erase(std::remove(c.begin(), c.end(), 7), c.end());
    return c;
}

std::string tune_key(const BatchSpec& sp, const std::vector<int>& idx) {
    std::ostringstream s;
    s << "prec" << sp.o->precision << ":int" << sp.o->integrator << ":B" << sp.o->n_traj << ":lags"
      << (sp.L > 0 ? 1 : 0) << ":N";
    for (size_t q = 0; q < idx.size(); ++q) s << (q ? "," : "") << sp.pts[idx[q]].N;
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

// times a few plain steps of the bucket's points alone for every candidate
int autotune_bucket(const BatchSpec& sp, const std::vector<int>& idx, int bucket, hipStream_t st, int* best_cfg) {
    *best_cfg = -1;
    double best_ms = 1e300;
    const StepKind plain{false, false, false, false};
    for (int cfg : bucket_candidates(bucket, sp.o->precision)) {
        std::vector<Bucket> one(1);
        one[0].stream = st;
        BatchSpec sp0 = sp;
        sp0.L = 0;   // the plain step decides
        int rc = build_bucket(sp0, idx, cfg, one[0], st);
        if (rc == TWA_OK) {
            std::vector<hipEvent_t> ev;
            rc = bucket_step(one[0], 0, plain, st);   // warm-up
            hipEvent_t a, b;
            hipEventCreate(&a);
            hipEventCreate(&b);
            hipEventRecord(a, st);
            int cur = 1;
            for (int s = 0; s < 4 && rc == TWA_OK; ++s) {
                rc = bucket_step(one[0], cur, plain, st);
                cur = 1 - cur;
            }
            hipEventRecord(b, st);
            hipStreamSynchronize(st);
            float ms = 0.f;
            hipEventElapsedTime(&ms, a, b);
            hipEventDestroy(a);
            hipEventDestroy(b);
            if (rc == TWA_OK && ms < best_ms) {
                best_ms = ms;
                *best_cfg = cfg;
            }
        }
        one[0].release();
        if (rc == TWA_ENOMEM) continue;
        if (rc != TWA_OK) return rc;
    }
    if (*best_cfg < 0) {
        set_error("twa_run_batch: no tile configuration fits");
        return TWA_ENOMEM;
    }
    return TWA_OK;
}

}  // namespace

int run_batch(const twa_point* pts, int np, const twa_batch_opts* o, twa_observables* outs) {
    if (!pts || np < 1 || !o || !outs || o->n_traj < 1 || o->n_steps < 1 || !(o->gamma > 0)) {
        set_error("twa_run_batch: need points, options, outputs, n_traj >= 1, n_steps >= 1, gamma > 0");
        return TWA_EINVAL;
    }
    if (o->integrator != TWA_INT_HEUN && o->integrator != TWA_INT_SIB) {
        set_error("twa_run_batch: integrator must be TWA_INT_HEUN or TWA_INT_SIB");
        return TWA_EINVAL;
    }
    if (o->precision != TWA_PREC_FP64 && o->precision != TWA_PREC_FP32 && o->precision != TWA_PREC_BF16 &&
        o->precision != TWA_PREC_FP16 && o->precision != TWA_PREC_BF16X3) {
        set_error("twa_run_batch: precision must be FP64, FP32, BF16, FP16 or split BF16");
        return TWA_EINVAL;
    }
    if (o->tile_config >= 0 && ((o->tile_config > 3 && o->tile_config != 7) ||
                                (o->tile_config == 7 && o->precision == TWA_PREC_FP64))) {
        set_error("twa_run_batch: tile_config must be 0..3 or 7 (not 7 in FP64)");
        return TWA_EINVAL;
    }
    for (int p = 0; p < np; ++p)
        if (pts[p].N < 1 || !(pts[p].dt > 0) || !std::isfinite(pts[p].dt) || !std::isfinite(pts[p].w) ||
            !std::isfinite(pts[p].alpha) || pts[p].w < 0 || pts[p].alpha < 0) {
            set_error("twa_run_batch: point " + std::to_string(p) + " is invalid");
            return TWA_EINVAL;
        }
    const int64_t burnin = o->burnin < 0 ? o->n_steps / 2 : o->burnin;
    if (burnin >= o->n_steps) {
        set_error("twa_run_batch: the averaging window is empty");
        return TWA_EINVAL;
    }
    const int64_t L = std::max<int64_t>(0, o->n_lags);
    int64_t stride = 1;
    if (L > 0) {
        if (o->integrator != TWA_INT_HEUN) {
            set_error("twa_run_batch: the two-time response copies are defined for the Heun integrator");
            return TWA_EINVAL;
        }
        stride = o->lag_stride > 0 ? o->lag_stride : std::max<int64_t>(1, (o->n_steps - burnin) / L);
        if ((L - 1) * stride > o->n_steps - burnin) {
            set_error("twa_run_batch: (n_lags - 1) * lag_stride exceeds the window");
            return TWA_EINVAL;
        }
    }
    hipStream_t st = (hipStream_t)o->stream;
    hipStream_t own = nullptr;
    if (!st) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) {
            set_error("twa_run_batch: hipStreamCreate failed (no usable GPU?)");
            return TWA_EHIP;
        }
        st = own;
    }
    std::vector<twa_pump*> pumps((size_t)np, nullptr);
    std::vector<Bucket> bks;
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> ev;
    GraphSet gset;
    int rc = TWA_OK;
    int cur = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float loop_ms = 0.f;
    std::string err_msg;
    const int GS = o->steps_per_graph > 0 ? (o->steps_per_graph + 1) / 2 * 2 : 16;
    BatchSpec sp{pts, o, &pumps, burnin, L, stride};
    Plan plan{burnin, L, stride, burnin + (L > 0 ? (L - 1) * stride : 0)};
    const int J = (int)std::min<int64_t>(32, o->n_traj);
    for (int p = 0; p < np && rc == TWA_OK; ++p) rc = twa_build_pump(pts[p].N, pts[p].w, pts[p].alpha, &pumps[(size_t)p]);
    if (rc) goto cleanup;
    {
        // buckets: one tile configuration per N bucket (or one given for all)
        std::vector<std::vector<int>> groups(3);
        for (int p = 0; p < np; ++p) groups[(size_t)(o->tile_config >= 0 ? 0 : bucket_of(pts[p].N))].push_back(p);
        for (int b = 0; b < 3; ++b) {
            if (groups[(size_t)b].empty()) continue;
            int cfg = o->tile_config;
            if (cfg < 0) {
                const std::string key = tune_key(sp, groups[(size_t)b]);
                cfg = cached_cfg(o->tune_cache, key);
                const std::vector<int> cand = bucket_candidates(b, o->precision);
                if (std::find(cand.begin(), cand.end(), cfg) == cand.end()) {
                    if ((rc = autotune_bucket(sp, groups[(size_t)b], b, st, &cfg))) goto cleanup;
                    store_cfg(o->tune_cache, key, cfg);
                }
            }
            bks.emplace_back();
            if ((rc = build_bucket(sp, groups[(size_t)b], cfg, bks.back(), st))) goto cleanup;
        }
        branch.assign(bks.size(), nullptr);
        ev.assign(bks.size() + 1, nullptr);
        for (auto& e : ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                set_error("twa_run_batch: hipEventCreate failed");
                rc = TWA_EHIP;
                goto cleanup;
            }
        for (size_t b = 0; b < bks.size(); ++b) {
            if (bks.size() > 1) {
                if (hipStreamCreateWithFlags(&branch[b], hipStreamNonBlocking) != hipSuccess) {
                    set_error("twa_run_batch: hipStreamCreate failed");
                    rc = TWA_EHIP;
                    goto cleanup;
                }
                bks[b].stream = branch[b];
            } else {
                bks[b].stream = st;
            }
        }
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("twa_run_batch: set-up failed");
        rc = TWA_EHIP;
        goto cleanup;
    }
    hipEventRecord(e0, st);
    if ((rc = run_steps(bks, plan, 0, o->n_steps, cur, o->use_graph != 0, GS, o->progress_every, st, ev, gset)))
        goto cleanup;
    hipEventRecord(e1, st);
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("twa_run_batch: step kernels failed");
        rc = TWA_EHIP;
        goto cleanup;
    }
    hipEventElapsedTime(&loop_ms, e0, e1);
    for (auto& bk : bks)
        for (size_t q = 0; q < bk.gs.size(); ++q) {
            const int p = bk.idx[q];
            const Geometry& g = bk.gs[q];
            const EnsembleBuffers& b = bk.bs[q];
            const twa_outputs* po = o->outputs ? &o->outputs[p] : nullptr;
            const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (g.B * g.N + 255) / 256));
            if ((rc = launch_finish(g, b, cur, nb, st))) goto cleanup;
            const size_t se = (size_t)state_elt_bytes(g.precision);
            std::vector<char> momraw((size_t)10 * g.Bp * se);
            std::vector<float> diag((size_t)2 * nb);
            std::vector<double> hlag((size_t)L * J * 6);
            bool ok = hipMemcpyAsync(momraw.data(), b.mom, momraw.size(), hipMemcpyDeviceToHost, st) == hipSuccess &&
                      hipMemcpyAsync(diag.data(), b.diag, diag.size() * sizeof(float), hipMemcpyDeviceToHost, st) ==
                          hipSuccess;
            if (ok && L > 0)
                ok = hipMemcpyAsync(hlag.data(), b.lag, hlag.size() * sizeof(double), hipMemcpyDeviceToHost, st) ==
                     hipSuccess;
            double* export_dev = nullptr;
            if (ok && po && po->final_state) {
                ok = hipMalloc(&export_dev, (size_t)3 * g.B * g.N * sizeof(double)) == hipSuccess &&
                     launch_export_state(g, b.s[cur], export_dev, st) == TWA_OK &&
                     hipMemcpyAsync(po->final_state, export_dev, (size_t)3 * g.B * g.N * sizeof(double),
                                    hipMemcpyDeviceToHost, st) == hipSuccess;
            }
            ok = ok && hipStreamSynchronize(st) == hipSuccess;
            hipFree(export_dev);
            if (!ok) {
                set_error("twa_run_batch: copy-back failed");
                rc = TWA_EHIP;
                goto cleanup;
            }
            const int64_t ns = o->n_steps - burnin;
            std::vector<double> traj((size_t)g.B * 5);
            bool nan = false;
            for (int64_t k = 0; k < g.B; ++k)
                for (int m = 0; m < 5; ++m) {
                    double s, c;
                    if (se == 8) {
                        s = reinterpret_cast<const double*>(momraw.data())[(size_t)(2 * m) * g.Bp + k];
                        c = reinterpret_cast<const double*>(momraw.data())[(size_t)(2 * m + 1) * g.Bp + k];
                    } else {
                        s = reinterpret_cast<const float*>(momraw.data())[(size_t)(2 * m) * g.Bp + k];
                        c = reinterpret_cast<const float*>(momraw.data())[(size_t)(2 * m + 1) * g.Bp + k];
                    }
                    const double v = (s - c) / (double)ns;
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
            out.n_lags = L;
            out.lag_stride = stride;
            out.max_norm_dev = mx;
            out.step_criterion = std::max(o->gamma * (double)g.N, pumps[(size_t)p]->lam_max) * pts[p].dt;
            out.nan_flag = nan ? 1 : 0;
            out.tile_config = bk.cfg;
            out.kernel_ms = loop_ms;   // the whole scan's step loop
            const double nnb = (double)g.N * (double)g.N * (double)g.B;
            out.gemm_flops = 12.0 * nnb * (double)o->n_steps + (L > 0 ? 16.0 * nnb * (double)((L - 1) * stride) : 0.0);
            out.linewidth = NAN;
            out.linewidth_sym = NAN;
            out.I_gen = out.g2_gen = out.I_gen_se = out.g2_gen_se = NAN;
            if (L > 0) finalize_lags(hlag, L, J, g.B, stride, pts[p].dt, o->kappa, &out, po);
            if (po && po->traj_moments) std::memcpy(po->traj_moments, traj.data(), traj.size() * sizeof(double));
            if (po && po->n_blocks) *po->n_blocks = J;
            const int st_p =
                run_status(("twa_run_batch: point " + std::to_string(p)).c_str(), nan, mx, o->norm_tol);
            if (st_p != TWA_OK && rc == TWA_OK) {
                rc = st_p;
                err_msg = twa_last_error();
            }
        }
    if (rc == TWA_EUNSTABLE) set_error(err_msg);
cleanup:
    if (rc != TWA_OK && rc != TWA_EUNSTABLE) hipStreamSynchronize(st);
    for (auto& b : branch)
        if (b) hipStreamSynchronize(b);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    for (auto& e : ev)
        if (e) hipEventDestroy(e);
    for (auto& bk : bks) bk.release();
    for (auto& b : branch)
        if (b) hipStreamDestroy(b);
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
    o->norm_tol = 1e-2;
    o->n_lags = 0;
    o->lag_stride = 0;
    o->kappa = 0.25;
    o->tile_config = -1;
    o->progress_every = 0;
    o->outputs = nullptr;
}

TWA_API int twa_run_batch(const twa_point* pts, int n_points, const twa_batch_opts* o, twa_observables* outs) {
    TWA_API_LOCK();
    return twa::run_batch(pts, n_points, o, outs);
}

}  // extern "C"
