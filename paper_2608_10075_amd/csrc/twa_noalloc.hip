// twa_run_noalloc: twa_run for callers that cannot allocate device memory
// (tight serving loops, harnesses that forbid allocation).  It ends with a
// copy of the results to the host and a synchronisation of the caller's
// stream, so it is not itself capturable into a hipGraph.  Every buffer of
// the run is carved from one file-scope device
// array of fixed size, `scratch`; the kernels are those of twa_run, so the
// results are the same bit for bit.  The per-trajectory window averages are
// reduced to jackknife block sums on the device, so the host side needs no
// allocation either.
//
// Each device the library runs on holds its own copy of `scratch` until the
// process ends; its address on a device is taken once, with that device
// current, by hipGetSymbolAddress (the name of the array in host code is only
// a host-side stand-in).  Every call on a device uses the same array: calls
// that overlap on one device race.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "twa_device.h"
#include "twa_internal.h"
#include "twa_run.h"

namespace twa {

namespace {

__device__ __align__(256) unsigned char scratch[TWA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current device (resolved on first use)
int scratch_address(void** out) {
    int dev = 0;
    TWA_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("twa_run_noalloc: device index out of range");
        return TWA_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("twa_run_noalloc: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return TWA_EHIP;
        }
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return TWA_OK;
}

// bump allocation inside the scratch array (256-byte aligned pieces)
struct Carver {
    char* base;
    size_t used = 0;
    void* take(size_t bytes) {
        void* p = base + used;
        used += (std::max<size_t>(bytes, 16) + 255) / 256 * 256;
        return p;
    }
};

__global__ void zero_kernel(uint4* p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = uint4{0u, 0u, 0u, 0u};
}

// jackknife block sums of the per-trajectory window averages
// (mom: Kahan (sum, compensation) pairs [5][2][Bp]), summed in trajectory
// order within a block as the host finaliser of twa_run does; res[J*5 + 0]
// = 1 if any average is not finite.  Also res[J*5 + 1] = max of the
// end-of-run norm deviations diag[0 .. nblk), res[J*5 + 2] = 1 if any block
// saw a non-finite state.
template <typename S>
__global__ __launch_bounds__(256) void block_sums_kernel(const S* mom, int64_t B, int64_t Bp, int J, int64_t ns,
                                                         const float* diag, int nblk, double* res) {
    const int t = threadIdx.x;
    __shared__ int bad;
    if (t == 0) bad = 0;
    __syncthreads();
    if (t < J * 5) {
        const int j = t / 5, m = t % 5;
        const int64_t klo = ((int64_t)j * B + J - 1) / J, khi = ((int64_t)(j + 1) * B + J - 1) / J;
        double acc = 0;
        for (int64_t k = klo; k < khi; ++k) {
            const double s = (double)mom[(2 * m) * Bp + k], c = (double)mom[(2 * m + 1) * Bp + k];
            const double v = (s - c) / (double)ns;
            if (!isfinite(v)) bad = 1;
            acc += v;
        }
        res[t] = acc;
    }
    __syncthreads();
    if (t == 0) {
        double mx = 0;
        int nan = 0;
        for (int i = 0; i < nblk; ++i) {
            mx = fmax(mx, (double)diag[i]);
            if (diag[nblk + i] != 0.f) nan = 1;
        }
        res[J * 5 + 0] = bad ? 1.0 : 0.0;
        res[J * 5 + 1] = mx;
        res[J * 5 + 2] = nan ? 1.0 : 0.0;
    }
}

}  // namespace

int run_noalloc(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                twa_observables* out) {
    if (!p || !p->pump || !out || n_traj < 1 || n_steps < 1 || !(dt > 0) || !std::isfinite(dt) ||
        !(p->gamma > 0) || !std::isfinite(p->gamma) ||
        (p->integrator != TWA_INT_HEUN && p->integrator != TWA_INT_SIB)) {
        set_error("twa_run_noalloc: need params with a pump, n_traj >= 1, n_steps >= 1, dt > 0, gamma > 0, "
                  "integrator TWA_INT_HEUN or TWA_INT_SIB");
        return TWA_EINVAL;
    }
    const twa_pump* pump = p->pump;
    if (!pump->W || pump->G || pump->Om || p->pump_path != TWA_PUMP_DENSE || p->n_lags > 0 || p->init_state ||
        p->precision < TWA_PREC_FP64 || p->precision > TWA_PREC_BF16X3) {
        set_error("twa_run_noalloc: a dense pump (twa_build_pump or twa_build_pump_dense), no lags, no initial "
                  "state, a known precision");
        return TWA_EINVAL;
    }
    const int64_t N = pump->N, B = n_traj;
    const int64_t burnin = p->burnin < 0 ? n_steps / 2 : p->burnin;
    if (burnin >= n_steps) {
        set_error("twa_run_noalloc: the averaging window is empty");
        return TWA_EINVAL;
    }
    const int cfg = p->tile_config >= 0 ? p->tile_config : pick_tile_cfg(p->precision, N, B);
    if (cfg >= n_tile_cfgs() || (p->precision == TWA_PREC_FP64 && cfg > 3)) {
        set_error("twa_run_noalloc: unknown tile configuration");
        return TWA_EINVAL;
    }
    Geometry g = make_geometry(p->precision, cfg, N, B);
    g.integrator = p->integrator;
    const bool fused = p->tile_config < 0 && small_path_applies(p->precision, N, 0);
    const int J = (int)std::min<int64_t>(32, B);
    const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (B * N + 255) / 256));
    hipStream_t st = (hipStream_t)p->stream;

    // the buffers twa_run allocates for a run without lags, in the scratch array
    const size_t ge = (size_t)gemm_elt_bytes(g.precision), se = (size_t)state_elt_bytes(g.precision);
    const size_t P = (size_t)g.P, Bp = (size_t)g.Bp, C2 = (size_t)g.C2, nmt = (size_t)g.nmt;
    const size_t spl = (size_t)operand_split(g.precision);
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    Carver cv{static_cast<char*>(base)};
    EnsembleBuffers b;
    b.A = cv.take(P * 2 * P * ge * spl);
    b.Xop = cv.take(C2 * 2 * P * ge * spl);
    b.Dop = cv.take(C2 * P * ge * spl);
    b.s[0] = cv.take(3 * Bp * P * se);
    b.s[1] = cv.take(3 * Bp * P * se);
    b.Sn = cv.take(2 * Bp * se);
    b.Y = cv.take(2 * Bp * P * se);
    b.part[0] = cv.take(3 * nmt * Bp * se);
    b.part[1] = cv.take(3 * nmt * Bp * se);
    b.g = cv.take(2 * Bp * se);
    b.norm0 = cv.take(Bp * P * se);
    b.mom = cv.take(10 * Bp * se);
    b.step = static_cast<int64_t*>(cv.take(sizeof(int64_t)));
    b.diag = static_cast<float*>(cv.take(2 * 1024 * sizeof(float)));
    double* res = static_cast<double*>(cv.take((32 * 5 + 3) * sizeof(double)));
    if (cv.used > (size_t)TWA_NOALLOC_SCRATCH_BYTES) {
        set_error("twa_run_noalloc: N = " + std::to_string(N) + ", n_traj = " + std::to_string(B) + " needs " +
                  std::to_string(cv.used) + " bytes of device scratch; the limit is " +
                  std::to_string((size_t)TWA_NOALLOC_SCRATCH_BYTES) + " (use twa_run)");
        return TWA_ENOMEM;
    }

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
    // the previous call's contents stay in the array: clear what this run uses
    // (the buffers start at zero in twa_run), with a kernel rather than a memset
    {
        const size_t n16 = cv.used / 16;
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)std::min<size_t>(4096, (n16 + 255) / 256)), dim3(256), 0, st,
                           static_cast<uint4*>(base), n16);
        TWA_HIP_CHECK(hipGetLastError());
    }
    if ((rc = launch_build_A(g, pump->W, pump->F, dt, b.A, st))) return rc;
    if ((rc = launch_init_state(g, b, c, nullptr, st))) return rc;
    if ((rc = launch_reduce_state(g, b.s[0], b.part[0], st))) return rc;
    int cur = 0;
    if (fused) {
        cur = (int)(n_steps & 1);
        if ((rc = launch_small_run(g, b, c, pump, dt, n_steps, cur, st))) return rc;
    } else {
        for (int64_t n = 0; n < n_steps; ++n) {
            if ((rc = launch_step_kernels(g, b, c, cur, false, nullptr, st))) return rc;
            if (n + 1 > burnin && (rc = launch_observe(g, b, c, 1 - cur, false, st))) return rc;
            cur = 1 - cur;
        }
    }
    if ((rc = launch_finish(g, b, cur, nblk, st))) return rc;
    const int64_t ns = n_steps - burnin;
    if (g.precision == TWA_PREC_FP64)
        hipLaunchKernelGGL(block_sums_kernel<double>, dim3(1), dim3(256), 0, st, static_cast<const double*>(b.mom), B,
                           g.Bp, J, ns, b.diag, nblk, res);
    else
        hipLaunchKernelGGL(block_sums_kernel<float>, dim3(1), dim3(256), 0, st, static_cast<const float*>(b.mom), B,
                           g.Bp, J, ns, b.diag, nblk, res);
    TWA_HIP_CHECK(hipGetLastError());
    double hres[32 * 5 + 3];
    TWA_HIP_CHECK(hipMemcpyAsync(hres, res, (size_t)(J * 5 + 3) * sizeof(double), hipMemcpyDeviceToHost, st));
    TWA_HIP_CHECK(hipStreamSynchronize(st));
    double bcnt[32];
    for (int j = 0; j < J; ++j) {
        const int64_t klo = ((int64_t)j * B + J - 1) / J, khi = ((int64_t)(j + 1) * B + J - 1) / J;
        bcnt[j] = (double)(khi - klo);
    }
    std::memset(out, 0, sizeof(*out));
    finalize_blocks(hres, bcnt, J, B, out);
    const bool nan = hres[J * 5 + 0] != 0.0 || hres[J * 5 + 2] != 0.0;
    out->n_samples = ns;
    out->max_norm_dev = hres[J * 5 + 1];
    out->step_criterion = std::max(p->gamma * (double)N, pump->lam_max) * dt;
    out->nan_flag = nan ? 1 : 0;
    out->tile_config = fused ? TWA_TILE_FUSED : cfg;
    out->kernel_ms = NAN;
    out->gemm_flops = (double)n_steps * 12.0 * (double)N * (double)N * (double)B;
    out->linewidth = out->linewidth_sym = NAN;
    out->I_gen = out->g2_gen = out->I_gen_se = out->g2_gen_se = NAN;
    return run_status("twa_run_noalloc", nan, out->max_norm_dev, p->norm_tol);
}

}  // namespace twa

extern "C" {

TWA_API int twa_run_noalloc(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                            twa_observables* out) {
    TWA_API_LOCK();
    return twa::run_noalloc(p, n_traj, dt, n_steps, seed, out);
}

}  // extern "C"
