// Run driver of the C ABI: buffer management, the step loop (direct launches
// or replayed hipGraphs), and the host-side finalisation of the few kB of
// accumulators copied back once at the end (the paper's End Matter advises a
// single device-to-host transfer at the end of the simulation).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>

#include "twa_internal.h"
#include "twa_run.h"

namespace twa {

static thread_local std::string g_err;

std::recursive_mutex& api_mutex() {
    static std::recursive_mutex m;
    return m;
}
void set_error(const std::string& msg) { g_err = msg; }

int gemm_elt_bytes(int precision) {
    switch (precision) {
        case TWA_PREC_FP64: return 8;
        case TWA_PREC_FP32: return 4;
        default: return 2;
    }
}
int state_elt_bytes(int precision) { return precision == TWA_PREC_FP64 ? 8 : 4; }
int operand_split(int precision) { return precision == TWA_PREC_BF16X3 ? 3 : 1; }

int pick_tile_cfg(int precision, int64_t N, int64_t n_traj) {
    if (N <= 48) return 0;
    if (N <= 768) return 1;
    if (precision == TWA_PREC_FP64) return 2;
    // Large N: 128x128 tiles (4 waves) or 320x256 tiles (8 waves), whichever
    // gives the shorter estimated contraction time = rounds of resident tiles
    // x work per tile / per-tile rate.  The larger tile moves 45 % fewer bytes
    // per flop through the vector-memory path (the bound of the smaller one)
    // and runs 1.64x faster per tile, but needs enough tiles to fill the device.
    static int ncu = 0;
    if (ncu <= 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
    }
    auto est = [&](int cfg, double rate) {
        const TileCfg& t = tile_cfg(cfg);
        const int64_t P = round_up(N, t.mt), Bp = round_up(n_traj, t.nt / 2);
        const int64_t tiles = (P / t.mt) * (2 * Bp / t.nt);
        const int64_t rounds = (tiles + ncu - 1) / ncu;
        return (double)rounds * (double)(t.mt * t.nt) / rate;
    };
    return est(7, 1.64) < est(2, 1.0) ? 7 : 2;
}

// ---------------------------------------------------------------------------
// host finalisation
void finalize_moments(const std::vector<double>& traj, int64_t B, twa_observables* o) {
    // traj: [B][5] per-trajectory window averages
    const int J = (int)std::min<int64_t>(32, B);
    double bsum[32 * 5] = {0}, bcnt[32] = {0};
    for (int64_t k = 0; k < B; ++k) {
        const int j = (int)((k * J) / B);
        for (int m = 0; m < 5; ++m) bsum[(size_t)j * 5 + m] += traj[(size_t)k * 5 + m];
        bcnt[(size_t)j] += 1.0;
    }
    finalize_blocks(bsum, bcnt, J, B, o);
}

void finalize_blocks(const double* bsum, const double* bcnt, int J, int64_t B, twa_observables* o) {
    double tot[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < J; ++j)
        for (int m = 0; m < 5; ++m) tot[m] += bsum[(size_t)j * 5 + m];
    auto derive = [](const double* m, double* d) {
        const double T2 = m[0], T3 = m[1], T4 = m[2], Z = m[3], ZZ = m[4];
        const double spsm = T2 + 0.5 * Z;
        const double num = T4 + 2.0 * T3 - Z / 3.0 + 0.5 * ZZ - (4.0 / 3.0) * T2;
        d[0] = Z;
        d[1] = spsm;
        d[2] = num / (spsm * spsm);
    };
    double mean[8];
    for (int m = 0; m < 5; ++m) mean[m] = tot[m] / (double)B;
    derive(mean, mean + 5);
    double se[8];
    if (J >= 2) {
        double vals[32 * 8];
        for (int j = 0; j < J; ++j) {
            double* v = &vals[(size_t)j * 8];
            for (int m = 0; m < 5; ++m) v[m] = (tot[m] - bsum[(size_t)j * 5 + m]) / ((double)B - bcnt[(size_t)j]);
            derive(v, v + 5);
        }
        for (int c = 0; c < 8; ++c) {
            double mu = 0;
            for (int j = 0; j < J; ++j) mu += vals[(size_t)j * 8 + c];
            mu /= J;
            double ss = 0;
            for (int j = 0; j < J; ++j) {
                const double d = vals[(size_t)j * 8 + c] - mu;
                ss += d * d;
            }
            se[c] = std::sqrt((double)(J - 1) / J * ss);
        }
    } else {
        for (int c = 0; c < 8; ++c) se[c] = NAN;
    }
    o->T2 = mean[0]; o->T3 = mean[1]; o->T4 = mean[2]; o->Z = mean[3]; o->ZZ = mean[4];
    o->Sz = mean[5]; o->SpSm = mean[6]; o->g2 = mean[7];
    o->T2_se = se[0]; o->T3_se = se[1]; o->T4_se = se[2]; o->Z_se = se[3]; o->ZZ_se = se[4];
    o->Sz_se = se[5]; o->SpSm_se = se[6]; o->g2_se = se[7];
}

void finalize_decay(const std::vector<double>& traj, int64_t B, twa_observables* o) {
    // traj: [B][9] per-trajectory window averages of (E2, E2^2, E2 D, Q3, R, D^2, U, V, D);
    // intensity I = E2 + D/2 and the four-point function of SM Sec. S1 step 6, g2 = four-point / I^2
    const int J = (int)std::min<int64_t>(32, B);
    std::vector<double> bsum((size_t)J * 9, 0.0), bcnt((size_t)J, 0.0);
    for (int64_t k = 0; k < B; ++k) {
        const int j = (int)((k * J) / B);
        for (int m = 0; m < 9; ++m) bsum[(size_t)j * 9 + m] += traj[(size_t)k * 9 + m];
        bcnt[(size_t)j] += 1.0;
    }
    double tot[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < J; ++j)
        for (int m = 0; m < 9; ++m) tot[m] += bsum[(size_t)j * 9 + m];
    auto derive = [](const double* m, double* d) {
        const double E2 = m[0], E2E2 = m[1], E2D = m[2], Q3 = m[3], R = m[4], DD = m[5], U = m[6], V = m[7], D = m[8];
        const double inten = E2 + 0.5 * D;
        const double num = E2E2 + E2D + Q3 - R / 3.0 + 0.25 * (DD + U) - (4.0 / 3.0) * V;
        d[0] = inten;
        d[1] = num / (inten * inten);
    };
    double mean[9], dm[2];
    for (int m = 0; m < 9; ++m) mean[m] = tot[m] / (double)B;
    derive(mean, dm);
    o->I_gen = dm[0];
    o->g2_gen = dm[1];
    o->I_gen_se = o->g2_gen_se = NAN;
    if (J >= 2) {
        std::vector<double> vals((size_t)J * 2);
        for (int j = 0; j < J; ++j) {
            double v[9];
            for (int m = 0; m < 9; ++m) v[m] = (tot[m] - bsum[(size_t)j * 9 + m]) / ((double)B - bcnt[(size_t)j]);
            derive(v, &vals[(size_t)j * 2]);
        }
        double se[2];
        for (int c = 0; c < 2; ++c) {
            double mu = 0;
            for (int j = 0; j < J; ++j) mu += vals[(size_t)j * 2 + c];
            mu /= J;
            double ss = 0;
            for (int j = 0; j < J; ++j) {
                const double d = vals[(size_t)j * 2 + c] - mu;
                ss += d * d;
            }
            se[c] = std::sqrt((double)(J - 1) / J * ss);
        }
        o->I_gen_se = se[0];
        o->g2_gen_se = se[1];
    }
}

// iterative radix-2 FFT computing sum_l c_l e^{+2 pi i k l / n}
static void fft_pos(std::vector<std::complex<double>>& a) {
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = 2.0 * M_PI / (double)len;
        const std::complex<double> wl(std::cos(ang), std::sin(ang));
        for (size_t i = 0; i < n; i += len) {
            std::complex<double> w(1.0, 0.0);
            for (size_t j = 0; j < len / 2; ++j) {
                const std::complex<double> u = a[i + j], v = a[i + j + len / 2] * w;
                a[i + j] = u + v;
                a[i + j + len / 2] = u - v;
                w *= wl;
            }
        }
    }
}

// S(omega_k) = 2 tau Re sum_l c_l e^{i omega_k l tau}, trapezoid weights at the
// ends, omega_k = 2 pi k / (n tau) with n = 8 L; FWHM around the global peak.
double linewidth_of(const std::vector<std::complex<double>>& corr, double tau) {
    const size_t L = corr.size();
    if (L < 2) return NAN;
    const size_t n = 8 * L;
    std::vector<std::complex<double>> c(n, 0.0);
    for (size_t l = 0; l < L; ++l) c[l] = corr[l];
    c[0] *= 0.5;
    c[L - 1] *= 0.5;
    std::vector<double> S(n);
    if ((n & (n - 1)) == 0) {
        fft_pos(c);
        for (size_t k = 0; k < n; ++k) S[k] = 2.0 * tau * c[k].real();
    } else {
        for (size_t k = 0; k < n; ++k) {
            double acc = 0;
            for (size_t l = 0; l < L; ++l) {
                const double ph = 2.0 * M_PI * (double)((k * l) % n) / (double)n;
                acc += c[l].real() * std::cos(ph) - c[l].imag() * std::sin(ph);
            }
            S[k] = 2.0 * tau * acc;
        }
    }
    // reorder to ascending omega: k = n/2 .. n-1 are negative frequencies
    std::vector<double> om(n), Sp(n);
    const size_t half = n / 2;
    for (size_t q = 0; q < n; ++q) {
        const size_t k = (q + half + (n % 2)) % n;   // matches fftfreq ordering after argsort
        const long kk = (k < (n + 1) / 2) ? (long)k : (long)k - (long)n;
        om[q] = 2.0 * M_PI * (double)kk / ((double)n * tau);
        Sp[q] = S[k];
    }
    size_t kp = 0;
    for (size_t q = 1; q < n; ++q)
        if (Sp[q] > Sp[kp]) kp = q;
    const double hm = 0.5 * Sp[kp];
    size_t i = kp;
    while (i > 0 && Sp[i] > hm) --i;
    if (Sp[i] > hm) return NAN;
    const double left = om[i] + (hm - Sp[i]) * (om[i + 1] - om[i]) / (Sp[i + 1] - Sp[i]);
    size_t j = kp;
    while (j < n - 1 && Sp[j] > hm) ++j;
    if (Sp[j] > hm) return NAN;
    const double right = om[j - 1] + (hm - Sp[j - 1]) * (om[j] - om[j - 1]) / (Sp[j] - Sp[j - 1]);
    return right - left;
}

int run_status(const char* who, bool nan, double max_norm_dev, double norm_tol) {
    const double tol = effective_norm_tol(norm_tol);
    if (nan) {
        set_error(std::string(who) + ": non-finite values in the state or accumulators");
        return TWA_EUNSTABLE;
    }
    if (tol > 0 && !(max_norm_dev <= tol)) {
        char buf[192];
        std::snprintf(buf, sizeof(buf),
                      "%s: a spin length drifted by %.3g (max_norm_dev) > norm_tol %.3g; Eq. (S1) conserves "
                      "|s_i|^2 -- reduce dt or use the semi-implicit integrator",
                      who, max_norm_dev, tol);
        set_error(buf);
        return TWA_EUNSTABLE;
    }
    return TWA_OK;
}

void finalize_lags(const std::vector<double>& hlag, int64_t L, int J, int64_t B, int64_t stride, double dt,
                   double kappa, twa_observables* out, const twa_outputs* outs) {
    std::vector<std::complex<double>> corr((size_t)L), csym((size_t)L);
    for (int64_t l = 0; l < L; ++l) {
        double s[6] = {0, 0, 0, 0, 0, 0};
        for (int j = 0; j < J; ++j)
            for (int q = 0; q < 6; ++q) s[q] += hlag[((size_t)l * J + j) * 6 + q];
        for (int q = 0; q < 6; ++q) s[q] /= (double)B;
        const std::complex<double> cs(s[0], s[1]);
        // kappa * i * (xx + yy + i yx - i xy)
        const std::complex<double> resp(s[2] + s[5], s[3] - s[4]);
        csym[(size_t)l] = cs;
        corr[(size_t)l] = cs + std::complex<double>(0.0, kappa) * resp;
    }
    const double tau = (double)stride * dt;
    out->linewidth = linewidth_of(corr, tau);
    out->linewidth_sym = linewidth_of(csym, tau);
    if (outs && outs->corr_blocks)
        for (size_t q = 0; q < (size_t)L * J; ++q) {
            outs->corr_blocks[2 * q] = hlag[6 * q];
            outs->corr_blocks[2 * q + 1] = hlag[6 * q + 1];
        }
    if (outs && outs->chi_blocks)
        for (size_t q = 0; q < (size_t)L * J; ++q)
            for (int r = 0; r < 4; ++r) outs->chi_blocks[4 * q + r] = hlag[6 * q + 2 + r];
}

// ---------------------------------------------------------------------------
void free_buffers(EnsembleBuffers& b) {
    void* ptrs[] = {b.A,      b.Xop,    b.Dop,  b.s[0], b.s[1],    b.dlt,     b.Y,      b.part[0],
                    b.part[1], b.g,     b.norm0, b.mom, b.tXop,    b.tDop,    b.ts[0],  b.ts[1],
                    b.tdlt,   b.tY,     b.tpart[0], b.tpart[1], b.sm0, b.lag, b.step, b.diag, b.Sn,
                    b.AG,     b.AGG,    b.Zop,  b.GX,   b.UZ,      b.dg,      b.gmom,  b.A2};
    for (void* q : ptrs) hipFree(q);
    b = EnsembleBuffers();
}

// device allocation cleared on the run's stream (never the null stream: a
// null-stream operation would synchronise with streams that other threads
// may be capturing into graphs)
static int dalloc(void** p, size_t bytes, hipStream_t st) {
    if (bytes == 0) bytes = 16;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
        return TWA_ENOMEM;
    }
    if (hipMemsetAsync(*p, 0, bytes, st) != hipSuccess) {
        set_error("hipMemsetAsync failed");
        return TWA_EHIP;
    }
    return TWA_OK;
}

int alloc_buffers(const Geometry& g, bool tangents, int64_t L, int J, EnsembleBuffers& b, hipStream_t st) {
    const size_t ge = (size_t)gemm_elt_bytes(g.precision), se = (size_t)state_elt_bytes(g.precision);
    const size_t P = (size_t)g.P, Bp = (size_t)g.Bp, C2 = (size_t)g.C2, nmt = (size_t)g.nmt;
    int rc;
#define TWA_A(ptr, bytes) \
    if ((rc = dalloc((void**)&(ptr), (bytes), st)) != TWA_OK) return rc;
    const size_t spl = (size_t)operand_split(g.precision);   // split form: hi, lo, hi blocks
    const size_t ck = g.coh ? 1 : 0;                          // coherent exchange: one more K block
    TWA_A(b.A, P * (2 + ck) * P * ge * spl)
    TWA_A(b.Xop, C2 * (2 + ck) * P * ge * spl)
    TWA_A(b.Dop, C2 * (1 + ck) * P * ge * spl)
    if (ck) {
        TWA_A(b.A2, P * 2 * P * ge)
    }
    TWA_A(b.s[0], 3 * Bp * P * se)
    TWA_A(b.s[1], 3 * Bp * P * se)
    TWA_A(b.dlt, 3 * Bp * P * se)
    TWA_A(b.Sn, 2 * Bp * se)
    TWA_A(b.Y, 2 * Bp * P * se)
    TWA_A(b.part[0], 3 * nmt * Bp * se)
    TWA_A(b.part[1], 3 * nmt * Bp * se)
    TWA_A(b.g, 2 * Bp * se)
    TWA_A(b.norm0, Bp * P * se)
    TWA_A(b.mom, 10 * Bp * se)
    TWA_A(b.step, sizeof(int64_t))
    TWA_A(b.diag, 2 * 1024 * sizeof(float))
    TWA_A(b.sm0, 2 * Bp * se)
    if (L > 0) {
        TWA_A(b.lag, (size_t)L * J * 6 * sizeof(double))
    }
    if (tangents) {
        TWA_A(b.tXop, 2 * C2 * P * ge * spl)
        TWA_A(b.tDop, 2 * C2 * P * ge * spl)
        TWA_A(b.ts[0], 2 * 3 * Bp * P * se)
        TWA_A(b.ts[1], 2 * 3 * Bp * P * se)
        TWA_A(b.tdlt, 2 * 3 * Bp * P * se)
        TWA_A(b.tY, 2 * 2 * Bp * P * se)
        TWA_A(b.tpart[0], 2 * 3 * nmt * Bp * se)
        TWA_A(b.tpart[1], 2 * 3 * nmt * Bp * se)
    }
#undef TWA_A
    return TWA_OK;
}

int alloc_decay_buffers(const Geometry& g, EnsembleBuffers& b, hipStream_t st) {
    const size_t ge = (size_t)gemm_elt_bytes(g.precision), se = (size_t)state_elt_bytes(g.precision);
    const size_t P = (size_t)g.P, Bp = (size_t)g.Bp;
    int rc;
    if ((rc = dalloc(&b.AG, P * P * ge, st)) || (rc = dalloc(&b.AGG, P * P * ge, st)) ||
        (rc = dalloc(&b.Zop, Bp * P * ge, st)) || (rc = dalloc(&b.GX, 2 * Bp * P * se, st)) ||
        (rc = dalloc(&b.UZ, Bp * P * se, st)) || (rc = dalloc(&b.dg, P * se, st)) ||
        (rc = dalloc((void**)&b.gmom, 18 * Bp * sizeof(double), st)))
        return rc;
    return TWA_OK;
}

Geometry make_geometry(int precision, int cfg, int64_t N, int64_t B) {
    Geometry g;
    g.precision = precision;
    g.cfg = cfg;
    const TileCfg& tc = tile_cfg(cfg);
    g.kt = tc.kbytes / gemm_elt_bytes(precision);
    g.N = N;
    g.B = B;
    g.P = round_up(N, std::max<int64_t>(tc.mt, g.kt));
    g.Bp = round_up(B, tc.nt / 2);
    g.nmt = g.P / tc.mt;
    g.C2 = 2 * g.Bp;
    return g;
}

}  // namespace twa

// ===========================================================================
extern "C" {

TWA_API const char* twa_last_error(void) { return twa::g_err.c_str(); }
TWA_API const char* twa_version(void) { return "twa-mi355x 0.1 (gfx950)"; }

TWA_API void twa_params_default(twa_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->gamma = 1.0;
    p->s0z = 1.0;
    p->burnin = -1;
    p->integrator = TWA_INT_HEUN;
    p->precision = TWA_PREC_FP32;
    p->n_lags = 0;
    p->lag_stride = 0;
    p->point = 0;
    p->tile_config = -1;
    p->stream = nullptr;
    p->init_state = nullptr;
    p->timing = 0;
    p->use_graph = 1;
    p->kappa = 0.25;
    p->adjoint_objectives = 0;
    p->pump_path = TWA_PUMP_DENSE;
    p->norm_tol = 1e-2;
}

TWA_API int twa_philox(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* out, void* stream) {
    TWA_API_LOCK();
    if (n < 0 || (n > 0 && (!ctr || !out))) {
        twa::set_error("twa_philox: bad arguments");
        return TWA_EINVAL;
    }
    int rc = twa::launch_philox(ctr, n, key0, key1, out, (hipStream_t)stream);
    if (rc) return rc;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
        twa::set_error("twa_philox: kernel failed");
        return TWA_EHIP;
    }
    return TWA_OK;
}

TWA_API int twa_noise(uint64_t seed, int64_t step, int32_t point, int64_t n_traj, int64_t N, int32_t fp64,
                      double* zeta, double* g, void* stream) {
    TWA_API_LOCK();
    if (n_traj < 1 || N < 1 || step < 0 || !zeta || !g) {
        twa::set_error("twa_noise: bad arguments");
        return TWA_EINVAL;
    }
    int rc = twa::launch_noise_debug(seed, step, point, n_traj, N, fp64, zeta, g, (hipStream_t)stream);
    if (rc) return rc;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
        twa::set_error("twa_noise: kernel failed");
        return TWA_EHIP;
    }
    return TWA_OK;
}

TWA_API int twa_run(const twa_params* p, int64_t n_traj, double dt, int64_t n_steps, uint64_t seed,
                    twa_observables* out, const twa_outputs* outs) {
    TWA_API_LOCK();
    return twa::run_single(p, n_traj, dt, n_steps, seed, out, outs);
}

}  // extern "C"
