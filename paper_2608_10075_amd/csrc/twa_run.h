// Run-driver internals shared by the single-run, batched and adjoint paths.
#pragma once

#include <complex>
#include <vector>

#include "twa_internal.h"

namespace twa {

// HIP-event timing of the contraction launches, harvested in batches so that
// the number of live events stays bounded.
struct StepTimer {
    static constexpr int POOL = 256;
    std::vector<hipEvent_t> ev;
    int used = 0;
    bool open = false;
    double total_ms = 0.0;
    int64_t count = 0;
    int init() {
        ev.resize(2 * POOL);
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) return TWA_EHIP;
        return TWA_OK;
    }
    void begin(hipStream_t st) {
        if (used == POOL) harvest(st);
        hipEventRecord(ev[2 * used], st);
        open = true;
    }
    void end(hipStream_t st) {
        if (!open) return;
        hipEventRecord(ev[2 * used + 1], st);
        ++used;
        open = false;
    }
    void harvest(hipStream_t st) {
        hipStreamSynchronize(st);
        for (int i = 0; i < used; ++i) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
            total_ms += ms;
            ++count;
        }
        used = 0;
    }
    ~StepTimer() {
        for (auto& e : ev)
            if (e) hipEventDestroy(e);
    }
};

// spin-length check of a run: the threshold on max_norm_dev (0: the default
// 1e-2; < 0: no check), and the status and message of a finished run
inline double effective_norm_tol(double t) { return t == 0 ? 1e-2 : t; }
int run_status(const char* who, bool nan, double max_norm_dev, double norm_tol);

void free_buffers(EnsembleBuffers& b);
int alloc_buffers(const Geometry& g, bool tangents, int64_t L, int J, EnsembleBuffers& b, hipStream_t st);
Geometry make_geometry(int precision, int cfg, int64_t N, int64_t B);
void finalize_moments(const std::vector<double>& traj, int64_t B, twa_observables* o);
// the same from the jackknife block sums bsum [J][5] of the per-trajectory
// window averages (trajectory k in block k J / B, summed in k order) and the
// block sizes bcnt [J]; J <= 32, no allocation
void finalize_blocks(const double* bsum, const double* bcnt, int J, int64_t B, twa_observables* o);
void finalize_decay(const std::vector<double>& traj, int64_t B, twa_observables* o);
double linewidth_of(const std::vector<std::complex<double>>& corr, double tau);
// two-time finalisation: lag sums hlag [L][J][6] (block sums of the symmetric
// part and of the four response curves) -> out->linewidth, linewidth_sym and
// the optional corr_blocks / chi_blocks of outs
void finalize_lags(const std::vector<double>& hlag, int64_t L, int J, int64_t B, int64_t stride, double dt,
                   double kappa, twa_observables* out, const twa_outputs* outs);

// per-launch timers for the two contraction stages (primal)
struct GemmTimers {
    StepTimer s1, s2;
};

int launch_step_kernels(const Geometry& g, EnsembleBuffers& b, const StepConsts& c, int cur, bool tan_active,
                        GemmTimers* tm, hipStream_t st);
int run_single(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
               twa_observables* out, const twa_outputs* outs);
int run_noalloc(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                twa_observables* out);
int run_tangent_w(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                  twa_observables* out, double* grads);

}  // namespace twa
