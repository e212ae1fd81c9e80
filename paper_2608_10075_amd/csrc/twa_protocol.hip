// The paper's simulation protocol (main text, methods paragraph; SM Sec. S1)
// and its threshold quantities (main text, results): the step criterion
// max(Gamma N, lambda_max) dt < 0.05, the preparation time tau_s, the window
// tau = 5/Gamma, the normalised pump w~ = lambda_max/(Gamma N), the
// fixed-noise threshold search by safeguarded Newton steps with the pathwise
// gradient of twa_adjoint, and the g2_min scan over w~.  Host orchestration of
// the library's entry points; the arithmetic of the trajectories stays in the
// step kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "twa_internal.h"

namespace twa {
namespace {

// Dirichlet eta(s) = sum_{m >= 1} (-1)^(m-1) / m^s for real s > 0 by Borwein's
// alternating-series algorithm (P. Borwein, "An efficient algorithm for the
// Riemann zeta function", 1991): with d_k = n sum_{i <= k} (n+i-1)! 4^i /
// ((n-i)! (2i)!), eta(s) = -(1/d_n) sum_{k < n} (-1)^k (d_k - d_n) / (k+1)^s,
// error below 3 / (3 + sqrt 8)^n.
double dirichlet_eta(double s) {
    const int n = 40;
    double d[n + 1];
    double t = 1.0 / n;   // i = 0 term: (n-1)! / n!
    double acc = t;
    d[0] = n * acc;
    for (int i = 0; i < n; ++i) {
        t *= 4.0 * (double)(n + i) * (double)(n - i) / ((double)(2 * i + 1) * (double)(2 * i + 2));
        acc += t;
        d[i + 1] = n * acc;
    }
    double sum = 0.0;
    for (int k = 0; k < n; ++k) {
        const double term = (d[k] - d[n]) / std::pow((double)(k + 1), s);
        sum += (k % 2 == 0) ? term : -term;
    }
    return -sum / d[n];
}

int64_t steps_for(double t, double dt) { return (int64_t)std::ceil(t / dt - 1e-9); }

double objective_value(int obj, const twa_observables& o, int64_t N) {
    return obj == TWA_OBJ_G2 ? o.g2 : o.SpSm / (double)N;
}

}  // namespace
}  // namespace twa

extern "C" {

TWA_API int twa_protocol(const twa_pump* pump, double gamma, double cfl, int32_t finite_size, twa_protocol_t* out) {
    TWA_API_LOCK();
    using namespace twa;
    if (!pump || !out || !(gamma > 0) || !std::isfinite(gamma) || !(cfl > 0) || !(cfl < 0.05)) {
        set_error("twa_protocol: need a pump, an output, gamma > 0 and 0 < cfl < 0.05");
        return TWA_EINVAL;
    }
    if (!std::isfinite(pump->lam_min)) {
        set_error("twa_protocol: needs the channel rates of a dense pump (twa_build_pump or twa_build_pump_dense)");
        return TWA_EINVAL;
    }
    const double N = (double)pump->N;
    twa_protocol_t r;
    std::memset(&r, 0, sizeof(r));
    r.lam_min = pump->lam_min;
    r.lam_max = pump->lam_max;
    r.dt = cfl / std::max(gamma * N, pump->lam_max);
    if (finite_size) {
        if (!std::isfinite(pump->w) || !std::isfinite(pump->alpha) || !(pump->w > 0)) {
            set_error("twa_protocol: finite_size needs a pump of Eq. (2) with w > 0");
            return TWA_EINVAL;
        }
        const double e = 2.0 * dirichlet_eta(pump->alpha) - 1.0;
        if (!(e > 0)) {
            set_error("twa_protocol: 2 eta(alpha) - 1 <= 0 (alpha too small for the finite-size preparation time)");
            return TWA_EINVAL;
        }
        r.tau_s = 10.0 / (pump->w * e);
    } else if (pump->alpha < 1.0) {
        r.tau_s = 10.0 / gamma;
    } else {
        if (!(pump->lam_min > 0)) {
            set_error("twa_protocol: lambda_min <= 0");
            return TWA_EINVAL;
        }
        r.tau_s = 10.0 / pump->lam_min;
    }
    r.tau = 5.0 / gamma;
    r.n_prep = steps_for(r.tau_s, r.dt);
    r.n_window = steps_for(r.tau, r.dt);
    r.wt = pump->lam_max / (gamma * N);
    *out = r;
    return TWA_OK;
}

TWA_API void twa_threshold_opts_default(twa_threshold_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->objective = TWA_OBJ_G2;
    o->target = 1.08;
    o->w_lo = 0.0;
    o->w_hi = 0.0;
    o->tol_w = 1e-6;
    o->max_iter = 30;
    o->ckpt_every = 256;
    o->derivative = TWA_DERIV_FORWARD;
}

TWA_API int twa_find_threshold(int64_t N, double alpha, const twa_params* p, int64_t n_traj, double dt,
                               int64_t n_steps, uint64_t seed, const twa_threshold_opts* o, double* w_root,
                               double* f_root, int32_t* n_iter) {
    TWA_API_LOCK();
    using namespace twa;
    if (!p || !o || N < 1 || !(alpha >= 0) || !std::isfinite(alpha) || !(o->w_lo > 0) ||
        !(o->w_hi > o->w_lo) || !std::isfinite(o->w_hi) || !(o->tol_w > 0) || o->max_iter < 1 ||
        (o->derivative != TWA_DERIV_FORWARD && o->derivative != TWA_DERIV_ADJOINT) ||
        (o->objective != TWA_OBJ_G2 && o->objective != TWA_OBJ_SPSM_N) || !std::isfinite(o->target)) {
        set_error("twa_find_threshold: need params, options with 0 < w_lo < w_hi, tol_w > 0, max_iter >= 1 and a "
                  "known objective");
        return TWA_EINVAL;
    }
    twa_pump* base = nullptr;
    int rc = twa_build_pump(N, o->w_hi, alpha, &base);
    if (rc) return rc;
    const int ck = o->ckpt_every > 0 ? o->ckpt_every : 256;
    // objective - target at w; with the pathwise derivative if grad != nullptr
    auto eval = [&](double w, double* f, double* grad) -> int {
        twa_pump* pw = nullptr;
        int e = pump_scaled(base, w, &pw);
        if (e) return e;
        twa_params q = *p;
        q.pump = pw;
        // the reverse sweep carries only the objective searched for
        q.adjoint_objectives = o->objective == TWA_OBJ_G2 ? 2 : 1;
        twa_observables ob;
        std::memset(&ob, 0, sizeof(ob));
        if (grad && o->derivative == TWA_DERIV_ADJOINT) {
            double g[4] = {0, 0, 0, 0};
            e = twa_adjoint(&q, n_traj, dt, n_steps, seed, ck, &ob, g);
            if (!e) *grad = o->objective == TWA_OBJ_G2 ? g[2] : g[0] / (double)N;
        } else if (grad) {
            double g[3] = {0, 0, 0};
            e = twa_tangent_w(&q, n_traj, dt, n_steps, seed, &ob, g);
            if (!e) *grad = o->objective == TWA_OBJ_G2 ? g[1] : g[0] / (double)N;
        } else {
            e = twa_run(&q, n_traj, dt, n_steps, seed, &ob, nullptr);
        }
        twa_pump_free(pw);
        if (!e) *f = objective_value(o->objective, ob, N) - o->target;
        return e;
    };
    double lo = o->w_lo, hi = o->w_hi, flo = 0, fhi = 0;
    int iters = 0;
    double x = 0, fx = 0;
    bool done = false;
    if ((rc = eval(lo, &flo, nullptr)) || (rc = eval(hi, &fhi, nullptr))) goto out;
    if (flo == 0 || fhi == 0) {
        x = flo == 0 ? lo : hi;
        fx = 0;
        done = true;
    } else if ((flo < 0) == (fhi < 0)) {
        set_error("twa_find_threshold: the objective does not cross the target on [w_lo, w_hi]");
        rc = TWA_ENOROOT;
        goto out;
    }
    // first point: where the chord through the bracket ends crosses the target
    x = lo - flo * (hi - lo) / (fhi - flo);
    while (!done && iters < o->max_iter) {
        double d = 0;
        if ((rc = eval(x, &fx, &d))) goto out;
        ++iters;
        if (fx == 0) {
            done = true;
            break;
        }
        if ((fx < 0) == (flo < 0)) {
            lo = x;
            flo = fx;
        } else {
            hi = x;
            fhi = fx;
        }
        double xn = (d != 0 && std::isfinite(d)) ? x - fx / d : 0.5 * (lo + hi);
        const bool newton_ok = xn > lo && xn < hi;
        if (!newton_ok) xn = 0.5 * (lo + hi);
        if ((newton_ok && std::fabs(xn - x) < o->tol_w) || hi - lo < o->tol_w) {
            done = true;   // x is within tol_w of the root
            break;
        }
        x = xn;
    }
    if (!done) {
        set_error("twa_find_threshold: no convergence within max_iter gradient evaluations");
        rc = TWA_ENOROOT;
    }
out:
    twa_pump_free(base);
    if (w_root) *w_root = x;
    if (f_root) *f_root = fx;
    if (n_iter) *n_iter = iters;
    return rc;
}

TWA_API int twa_g2_min(int64_t N, double alpha, const twa_params* p, int64_t n_traj, uint64_t seed,
                       int32_t n_points, double wt_lo, double wt_hi, double cfl, int32_t finite_size,
                       double* wt_out, double* g2_out, double* wt_min, double* g2_min) {
    TWA_API_LOCK();
    using namespace twa;
    if (!p || N < 1 || n_points < 1 || !(wt_lo > 0) || !(wt_hi >= wt_lo) || !std::isfinite(wt_hi) ||
        !(p->gamma > 0)) {
        set_error("twa_g2_min: need params with gamma > 0, n_points >= 1 and 0 < wt_lo <= wt_hi");
        return TWA_EINVAL;
    }
    twa_pump* base = nullptr;
    int rc = twa_build_pump(N, 1.0, alpha, &base);   // lambda_max is linear in w at fixed alpha
    if (rc) return rc;
    double best = INFINITY, best_wt = NAN;
    for (int32_t j = 0; j < n_points && !rc; ++j) {
        const double wt = n_points == 1 ? wt_lo : wt_lo + (wt_hi - wt_lo) * j / (double)(n_points - 1);
        const double w = wt * p->gamma * (double)N / base->lam_max;
        twa_pump* pw = nullptr;
        if ((rc = pump_scaled(base, w, &pw))) break;
        twa_protocol_t pr;
        rc = twa_protocol(pw, p->gamma, cfl, finite_size, &pr);
        if (!rc) {
            twa_params q = *p;
            q.pump = pw;
            q.burnin = pr.n_prep;
            twa_observables ob;
            std::memset(&ob, 0, sizeof(ob));
            rc = twa_run(&q, n_traj, pr.dt, pr.n_prep + pr.n_window, seed, &ob, nullptr);
            if (!rc) {
                if (wt_out) wt_out[j] = wt;
                if (g2_out) g2_out[j] = ob.g2;
                if (ob.g2 < best) {
                    best = ob.g2;
                    best_wt = wt;
                }
            }
        }
        twa_pump_free(pw);
    }
    twa_pump_free(base);
    if (!rc) {
        if (wt_min) *wt_min = best_wt;
        if (g2_min) *g2_min = best;
    }
    return rc;
}

}  // extern "C"
