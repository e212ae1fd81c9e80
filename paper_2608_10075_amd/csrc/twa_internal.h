// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/twa.h"

namespace twa {

// ---------------------------------------------------------------------------
// error plumbing
void set_error(const std::string& msg);

// Every entry point that touches the device holds this process-wide lock for
// its whole duration (recursive: the threshold search and the batch call
// other entry points).  hipFree synchronises the whole device, and a
// device-wide synchronisation while another thread's stream is being
// captured into a graph breaks that capture; serialising the calls keeps
// every free, allocation and pump build of one call out of another call's
// graph capture.
std::recursive_mutex& api_mutex();
#define TWA_API_LOCK() std::lock_guard<std::recursive_mutex> twa_api_lock_(::twa::api_mutex())
struct Status {
    int code = TWA_OK;
    std::string msg;
};
#define TWA_HIP_CHECK(expr)                                                       \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess) {                                                   \
            ::twa::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));  \
            return TWA_EHIP;                                                      \
        }                                                                         \
    } while (0)

// ---------------------------------------------------------------------------
// tile configurations of the channel-mixing contraction.  A configuration is
// (MT rows of spins, NT operand columns = NT/2 trajectories x 2 components,
// K bytes per LDS stage, waves along M, waves along N).
struct TileCfg {
    int id;
    int mt, nt, kbytes, waves_m, waves_n, nstage;
    const char* name;
};
int n_tile_cfgs();
const TileCfg& tile_cfg(int id);
int pick_tile_cfg(int precision, int64_t N, int64_t n_traj);

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
int gemm_elt_bytes(int precision);
int state_elt_bytes(int precision);
int operand_split(int precision);   // K blocks per operand value (3 for TWA_PREC_BF16X3)

// ---------------------------------------------------------------------------
// device buffers and launch geometry of one trajectory ensemble
struct Geometry {
    int precision;
    int cfg;
    int integrator = TWA_INT_HEUN;
    int coh = 0;         // coherent exchange: operand columns (s | zeta | s_perp), corrector [D | D_perp]
    int64_t N, B;        // atoms, trajectories
    int64_t P, Bp;       // padded
    int64_t nmt;         // P / MT
    int64_t C2;          // 2 * Bp operand columns
    int64_t kt;          // K elements per LDS stage
};

struct EnsembleBuffers {
    void* A = nullptr;          // GT [P][2P]  = [-dt/2 W | -sqrt(dt) F]
                                //    coherent exchange: [P][3P] = [-dt/2 W | -sqrt(dt) F | dt Omega]
    void* A2 = nullptr;         // GT [P][2P]  coherent exchange only: [-dt/2 W | dt Omega] (corrector)
    void* Xop = nullptr;        // GT [C2][2P] rows: (s^a | zeta^a) of one column; coherent exchange
                                //    [C2][3P] with s_perp = (s^y, -s^x) for the (x, y) columns
    void* Dop = nullptr;        // GT [C2][P]  predictor increments (coherent exchange [C2][2P]: D, D_perp)
    void* s[2] = {nullptr, nullptr};   // ST [3][Bp][P] ping-pong state
    void* dlt = nullptr;        // ST [3][Bp][P] predictor increment (kept only where response copies need it)
    void* Sn = nullptr;         // ST [2][Bp] collective sums S^x, S^y of the step's input state
    void* Y = nullptr;          // ST [2][Bp][P] contraction output of stage 1 (and 2)
    void* part[2] = {nullptr, nullptr};// ST [3][nmt][Bp] partial spin sums: [0] current state, [1] predictor
    void* g = nullptr;          // ST [2][Bp] collective normals of the step
    void* norm0 = nullptr;      // ST [Bp][P]
    void* mom = nullptr;        // ST [5][2][Bp] Kahan (sum, compensation)
    // response copies (two-time)
    void* tXop = nullptr;       // GT [2][C2][P]
    void* tDop = nullptr;       // GT [2][C2][P]
    void* ts[2] = {nullptr, nullptr};  // ST [2][3][Bp][P]
    void* tdlt = nullptr;       // ST [2][3][Bp][P]
    void* tY = nullptr;         // ST [2][2][Bp][P]
    void* tpart[2] = {nullptr, nullptr};// ST [2][3][nmt][Bp]
    void* sm0 = nullptr;        // ST [2][Bp]
    double* lag = nullptr;      // [L][J][6]
    // correlated decay (model handles)
    void* AG = nullptr;         // GT [P][P] G
    void* AGG = nullptr;        // GT [P][P] G o G (elementwise square)
    void* Zop = nullptr;        // GT [Bp][P] packed s^z operand
    void* GX = nullptr;         // ST [2][Bp][P] G s^x, G s^y
    void* UZ = nullptr;         // ST [Bp][P] (G o G) s^z
    void* dg = nullptr;         // ST [P] diagonal of G
    double* gmom = nullptr;     // [9][2][Bp] Kahan (sum, compensation) of the estimator quantities
    int64_t* step = nullptr;    // device step counter
    float* diag = nullptr;      // per-block max norm deviation / nan flags
};

struct StepConsts {
    double c1;      // Gamma dt / 2
    double c2;      // sqrt(Gamma dt)
    double s0z;
    uint32_t key0, key1;
    int32_t point;
    int64_t burnin, lag_stride, n_lags;
    int J;
};

// Type-erased description of one contraction launch (pointers are device
// buffers of the geometry's precision; kinds: 0 primal, 1 response tangent,
// 2 store (out = in + sign * A X), 3 adjoint of the corrector, 4 adjoint of
// the predictor, 5 semi-implicit, KIND_PRIMAL_WITH_Q the predictor that also
// stores the contribution of the second K half into Sout).
constexpr int KIND_PRIMAL_WITH_Q = 0x100;
struct GemmCall {
    int kind = 0, stage = 1, ncopy = 1;
    const void* A = nullptr;        // P rows, stage-blocked (a_index, the geometry's kt)
    const void* X = nullptr;
    int64_t ldx = 0, x_copy = 0, K = 0;
    double c1 = 0, c2 = 0;
    const void* s_cur = nullptr;
    void *s_next = nullptr, *dlt = nullptr, *Y = nullptr, *Y2out = nullptr, *Dop = nullptr, *Xnext = nullptr;
    int64_t ldxn = 0;
    const void* part_prim = nullptr;
    void* part_out = nullptr;
    const void* g = nullptr;
    int store_y2 = 0;
    const void* tpart_in = nullptr;
    int64_t* step = nullptr;
    const void* Sin = nullptr;
    void* Sout = nullptr;
    double store_sign = 1.0;
    const void *Y2in = nullptr, *Qin = nullptr, *YA = nullptr;
    void *lam = nullptr, *M1 = nullptr, *Rb = nullptr;
    double* gacc = nullptr;
    double inv_w = 0;
    // response / parameter tangent copies (kind 1): their state, increment,
    // field and operands; with Qin set, kind 1 adds the w-source Y/w - Q/(2w)
    const void* t_cur = nullptr;
    void *t_next = nullptr, *t_dlt = nullptr, *tY = nullptr, *tDop = nullptr;
    double srccoef[2][5] = {{0}};
    double src_scale = 0;
    int src_on = 0;
};
int launch_gemm_call(const Geometry& g, const GemmCall& c, hipStream_t st);

// Grouped persistent contraction launches over many ensembles that share a
// precision and tile configuration (one launch per stage covers all of them).
// Variants of a stage: the plain primal step, the primal step inside a
// two-time window (predictor increment kept, corrector field stored for the
// response copies) and the two response copies themselves.
enum { GV_PRIMAL = 0, GV_PRIMAL_TAN = 1, GV_TANGENT = 2, GV_COUNT = 3 };
struct GroupedPlan {
    void* d_args[GV_COUNT][2][2] = {};   // [variant][stage-1][cur] per-ensemble arguments
    int4* d_tiles[2] = {nullptr, nullptr};   // [0] (point, M tile, column tile, 0); [1] also copy 1
    int ntiles[2] = {0, 0};
    int grid[2] = {0, 0};
    int cfg = 0, precision = 0, integrator = TWA_INT_HEUN;
    bool tangents = false;
    int64_t* step = nullptr;
};
int grouped_prepare(const std::vector<Geometry>& gs, const std::vector<EnsembleBuffers>& bs,
                    const std::vector<StepConsts>& cs, int64_t* step, bool tangents, GroupedPlan& pl,
                    hipStream_t st);
// per-precision launchers, instantiated one precision per translation unit
// (twa_step_<precision>.hip); launch_gemm, launch_gemm_call, grouped_prepare
// and grouped_launch dispatch to them
template <int PREC>
int launch_gemm_p(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage, bool tangent, int cur,
                  bool store_y2, bool keep_dlt, hipStream_t st);
template <int PREC>
int launch_call_p(const Geometry& g, const GemmCall& c, hipStream_t st);
template <int PREC>
int grouped_prepare_p(const std::vector<Geometry>& gs, const std::vector<EnsembleBuffers>& bs,
                      const std::vector<StepConsts>& cs, int64_t* step, bool tangents, GroupedPlan& pl,
                      hipStream_t st);
template <int PREC>
int grouped_launch_p(const GroupedPlan& pl, int stage, int cur, int variant, hipStream_t st);
int grouped_launch(const GroupedPlan& pl, int stage, int cur, int variant, hipStream_t st);
void grouped_free(GroupedPlan& pl);

// kernel launchers (twa_step.hip, twa_aux.hip)
int launch_build_A(const Geometry& g, const double* W, const double* F, double dt, void* A, hipStream_t st);
int launch_build_A_coh(const Geometry& g, const double* W, const double* F, const double* Om, double dt, void* A,
                       void* A2, hipStream_t st);
int launch_init_state(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c,
                      const double* init_dev, hipStream_t st);
int launch_reduce_state(const Geometry& g, const void* s, void* part, hipStream_t st);
int launch_noise(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, hipStream_t st);
int launch_gemm(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage,
                bool tangent, int cur, bool store_y2, bool keep_dlt, hipStream_t st);
int launch_seed_tangents(const Geometry& g, const EnsembleBuffers& b, int cur, hipStream_t st);
int launch_observe(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int cur,
                   bool tangents, hipStream_t st);
int launch_finish(const Geometry& g, const EnsembleBuffers& b, int cur, int nblk, hipStream_t st);
int launch_export_state(const Geometry& g, const void* s, double* out_dev, hipStream_t st);
int launch_advance_step(int64_t* step, hipStream_t st);
int launch_philox(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t st);
int launch_noise_debug(uint64_t seed, int64_t step, int32_t point, int64_t B, int64_t N, int fp64,
                       double* zeta, double* g, hipStream_t st);

// fused small-N path (twa_small.hip): every step in one launch
bool small_path_applies(int precision, int64_t N, int64_t n_lags);
int launch_small_run(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const twa_pump* pump,
                     double dt, int64_t n_steps, int out_cur, hipStream_t st);

// correlated decay (twa_decay.hip): observation operands and the per-step
// estimator of correlated emission; the geometry pads trajectories to a
// multiple of the column tile
int decay_geometry_ok(const Geometry& g);
int alloc_decay_buffers(const Geometry& g, EnsembleBuffers& b, hipStream_t st);
int launch_decay_ops(const Geometry& g, const double* G, const EnsembleBuffers& b, hipStream_t st);
int launch_decay_observe(const Geometry& g, const EnsembleBuffers& b, int cur, hipStream_t st);

// Toeplitz fast path (twa_toeplitz.hip): circulant embedding of Eq. (2), one
// workgroup per trajectory over chunks of steps
int toeplitz_embedding_log2(int64_t N);
double toeplitz_spectrum_max(int64_t N, double w, double alpha);
int64_t toeplitz_max_n(int precision);
int toeplitz_tables(const Geometry& g, double w, double alpha, double dt, void** tw, void** spec, hipStream_t st);
int launch_toeplitz_run(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const void* tw,
                        const void* spec, int64_t n_steps, int cur, hipStream_t st);

// pump (twa_pump.hip): the Eq. (2) pump of a handle rescaled to amplitude w
int pump_scaled(const twa_pump* base, double w, twa_pump** out);
// sum over the nmt M-tile partials of trajectory k in tile order, for the
// channels c0 .. c0 + NC - 1; the loads of eight tiles are issued before
// their additions (the order of the additions is unchanged)
template <typename S, int NC>
__device__ __forceinline__ void tile_sums(const S* part, int64_t nmt, int64_t Bp, int64_t k, int c0, S (&out)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = 0;
    int64_t q = 0;
    for (; q + 8 <= nmt; q += 8) {
        S v[NC][8];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int u = 0; u < 8; ++u) v[c][u] = part[((c0 + c) * nmt + q + u) * Bp + k];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int u = 0; u < 8; ++u) out[c] += v[c][u];
    }
    for (; q < nmt; ++q)
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] += part[((c0 + c) * nmt + q) * Bp + k];
}

}  // namespace twa

struct twa_pump {
    int64_t N;
    double w, alpha;
    double lam_min, lam_max;
    double* W = nullptr;     // device FP64 [N][N]
    double* F = nullptr;     // device FP64 [N][N]
    double* V = nullptr;     // device FP64 eigenvectors, column-major (column j = vector j)
    double* lam = nullptr;   // host eigenvalues ascending [N]
    double* G = nullptr;     // device FP64 [N][N] correlated-decay matrix (model handles only); then
                             // W holds the drift matrix W - G and F, V, lam belong to W + G
    double* Om = nullptr;    // device FP64 [N][N] coherent exchange Omega (model handles, optional)
    int device = 0;
};
