// Pump matrix of Eq. (2), its channel decomposition (eigenvalues of w_ij, text
// after Eq. (2)) and the PSD square-root noise factor, all FP64 on the device.
// The eigendecomposition is a one-time setup step done with rocSOLVER's
// divide-and-conquer symmetric eigensolver; F = (V diag(sqrt(lambda+))) V^T
// with rocBLAS dgemm.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cfloat>
#include <cmath>
#include <vector>

#include "twa_internal.h"

namespace twa {

__global__ void pump_matrix_kernel(int64_t N, double w, double alpha, double* W) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t i = t / N, j = t % N;
    const double d = (double)(i > j ? i - j : j - i);
    W[t] = w / pow(d + 1.0, alpha);
}

__global__ void scale_columns_kernel(int64_t N, const double* V, const double* r, double* Vs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t col = t / N;   // column-major
    Vs[t] = V[t] * r[col];
}

__global__ void symmetrize_kernel(int64_t N, double* F) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t i = t / N, j = t % N;
    if (j <= i) return;
    const double v = 0.5 * (F[i * N + j] + F[j * N + i]);
    F[i * N + j] = v;
    F[j * N + i] = v;
}

// The builders work on a stream of their own, non-blocking, and synchronise
// only that stream: they never wait on, or make null-stream work wait on,
// streams that other threads may be capturing into graphs.
struct BuildStream {
    hipStream_t s = nullptr;
    BuildStream() = default;
    BuildStream(const BuildStream&) = delete;
    BuildStream& operator=(const BuildStream&) = delete;
    ~BuildStream() {
        if (s) hipStreamDestroy(s);
    }
    int create(const char* who) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            s = nullptr;
            set_error(std::string(who) + ": hipStreamCreateWithFlags failed (no usable GPU?)");
            return TWA_EHIP;
        }
        return TWA_OK;
    }
};

static int factorise(twa_pump* p, hipStream_t st) {
    const int64_t N = p->N;
    if (N > 46340) {
        set_error("N too large for a dense FP64 factorisation on one device");
        return TWA_EINVAL;
    }
    const size_t bytes = (size_t)N * N * sizeof(double);
    double *D = nullptr, *E = nullptr, *r = nullptr, *Vs = nullptr;
    rocblas_int* info = nullptr;
    rocblas_handle h = nullptr;
    int rc = TWA_OK;
    auto fail = [&](int code, const std::string& m) {
        set_error(m);
        rc = code;
    };
    std::vector<double> lam((size_t)N), rr((size_t)N);
    if (hipMalloc(&p->V, bytes) != hipSuccess || hipMalloc(&D, N * sizeof(double)) != hipSuccess ||
        hipMalloc(&E, N * sizeof(double)) != hipSuccess || hipMalloc(&r, N * sizeof(double)) != hipSuccess ||
        hipMalloc(&Vs, bytes) != hipSuccess || hipMalloc(&info, sizeof(rocblas_int)) != hipSuccess ||
        hipMalloc(&p->F, bytes) != hipSuccess) {
        fail(TWA_ENOMEM, "device allocation for the pump factorisation failed");
        goto done;
    }
    if (rocblas_create_handle(&h) != rocblas_status_success || rocblas_set_stream(h, st) != rocblas_status_success) {
        fail(TWA_EHIP, "rocblas_create_handle failed");
        goto done;
    }
    if (hipMemcpyAsync(p->V, p->W, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        fail(TWA_EHIP, "hipMemcpy failed");
        goto done;
    }
    // symmetric matrix: row- and column-major storage coincide
    if (rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)N, p->V, (rocblas_int)N, D, E,
                         info) != rocblas_status_success) {
        fail(TWA_EHIP, "rocsolver_dsyevd failed");
        goto done;
    }
    {
        rocblas_int hinfo = 0;
        if (hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(lam.data(), D, N * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            fail(TWA_EHIP, "hipMemcpy failed");
            goto done;
        }
        if (hinfo != 0) {
            fail(TWA_EHIP, "rocsolver_dsyevd did not converge");
            goto done;
        }
    }
    p->lam_min = lam[0];
    p->lam_max = lam[(size_t)N - 1];
    if (p->lam_min < -1e-10 * std::fabs(p->lam_max)) {
        fail(TWA_ENOTPSD, "pump matrix is not positive semidefinite");
        goto done;
    }
    {
        // eigenvalues within round-off of zero (rank-one alpha = 0) count as zero
        const double tol = 8.0 * (double)N * DBL_EPSILON * std::max(p->lam_max, 0.0);
        for (int64_t j = 0; j < N; ++j) rr[(size_t)j] = lam[(size_t)j] > tol ? std::sqrt(lam[(size_t)j]) : 0.0;
    }
    p->lam = (double*)malloc(N * sizeof(double));
    if (!p->lam) {
        fail(TWA_ENOMEM, "host allocation failed");
        goto done;
    }
    for (int64_t j = 0; j < N; ++j) p->lam[j] = lam[(size_t)j];
    if (hipMemcpyAsync(r, rr.data(), N * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess) {
        fail(TWA_EHIP, "hipMemcpy failed");
        goto done;
    }
    {
        const int64_t n2 = N * N;
        hipLaunchKernelGGL(scale_columns_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, N, p->V, r, Vs);
        const double one = 1.0, zero = 0.0;
        // column-major F = (V diag(sqrt(lambda+))) V^T
        if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)N, (rocblas_int)N,
                          (rocblas_int)N, &one, Vs, (rocblas_int)N, p->V, (rocblas_int)N, &zero, p->F,
                          (rocblas_int)N) != rocblas_status_success) {
            fail(TWA_EHIP, "rocblas_dgemm failed");
            goto done;
        }
        hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, N, p->F);
        if (hipStreamSynchronize(st) != hipSuccess) {
            fail(TWA_EHIP, "pump factorisation kernels failed");
            goto done;
        }
    }
done:
    hipStreamSynchronize(st);
    if (h) rocblas_destroy_handle(h);
    hipFree(D);
    hipFree(E);
    hipFree(r);
    hipFree(Vs);
    hipFree(info);
    return rc;
}

static void pump_release(twa_pump* p) {
    if (!p) return;
    hipFree(p->Om);
    hipFree(p->G);
    hipFree(p->W);
    hipFree(p->F);
    hipFree(p->V);
    free(p->lam);
    delete p;
}

__global__ void axpy_kernel(int64_t n, const double* a, double f, const double* b, double* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = a[t] + f * b[t];
}

static bool symmetric_finite(int64_t N, const double* M) {
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            const double a = M[i * N + j], b = M[j * N + i];
            if (!std::isfinite(a) || std::fabs(a - b) > 1e-12 * (std::fabs(a) + std::fabs(b))) return false;
        }
    return true;
}

__global__ void scale_kernel(int64_t n, const double* in, double f, double* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = f * in[t];
}

// The pump of Eq. (2) at amplitude w from one at amplitude w0 > 0 with the
// same alpha: W is linear in w and its PSD square root scales with sqrt(w),
// the eigenvectors are unchanged and the eigenvalues scale with w.
int pump_scaled(const twa_pump* b, double w, twa_pump** out) {
    if (!b || !out || !(b->w > 0) || !std::isfinite(b->w) || !(w > 0) || !std::isfinite(w) || !b->V || !b->lam) {
        set_error("pump_scaled: needs a pump from twa_build_pump with w > 0 and a target w > 0");
        return TWA_EINVAL;
    }
    const int64_t N = b->N, n2 = N * N;
    const double f = w / b->w;
    twa_pump* p = new twa_pump();
    p->N = N;
    p->w = w;
    p->alpha = b->alpha;
    p->lam_min = f * b->lam_min;
    p->lam_max = f * b->lam_max;
    p->device = b->device;
    const size_t bytes = (size_t)n2 * sizeof(double);
    if (hipMalloc(&p->W, bytes) != hipSuccess || hipMalloc(&p->F, bytes) != hipSuccess ||
        hipMalloc(&p->V, bytes) != hipSuccess) {
        pump_release(p);
        set_error("pump_scaled: device allocation failed");
        return TWA_ENOMEM;
    }
    p->lam = (double*)malloc((size_t)N * sizeof(double));
    if (!p->lam) {
        pump_release(p);
        set_error("pump_scaled: host allocation failed");
        return TWA_ENOMEM;
    }
    for (int64_t j = 0; j < N; ++j) p->lam[j] = f * b->lam[j];
    const unsigned nb = (unsigned)((n2 + 255) / 256);
    BuildStream bs;
    if (bs.create("pump_scaled")) {
        pump_release(p);
        return TWA_EHIP;
    }
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, bs.s, n2, b->W, f, p->W);
    hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, bs.s, n2, b->F, std::sqrt(f), p->F);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(p->V, b->V, bytes, hipMemcpyDeviceToDevice, bs.s) != hipSuccess ||
        hipStreamSynchronize(bs.s) != hipSuccess) {
        hipStreamSynchronize(bs.s);
        pump_release(p);
        set_error("pump_scaled: scaling failed");
        return TWA_EHIP;
    }
    *out = p;
    return TWA_OK;
}

}  // namespace twa

extern "C" {

TWA_API int twa_build_pump(int64_t N, double w, double alpha, twa_pump** out) {
    TWA_API_LOCK();
    using namespace twa;
    if (!out || N < 1 || !std::isfinite(w) || !std::isfinite(alpha) || w < 0 || alpha < 0) {
        set_error("twa_build_pump: need N >= 1, finite w >= 0, finite alpha >= 0 and an output pointer");
        return TWA_EINVAL;
    }
    *out = nullptr;
    twa_pump* p = new twa_pump();
    p->N = N;
    p->w = w;
    p->alpha = alpha;
    hipGetDevice(&p->device);
    if (hipMalloc(&p->W, (size_t)N * N * sizeof(double)) != hipSuccess) {
        delete p;
        set_error("twa_build_pump: device allocation failed");
        return TWA_ENOMEM;
    }
    const int64_t n2 = N * N;
    BuildStream bs;
    if (bs.create("twa_build_pump")) {
        pump_release(p);
        return TWA_EHIP;
    }
    hipLaunchKernelGGL(pump_matrix_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, bs.s, N, w, alpha, p->W);
    if (hipGetLastError() != hipSuccess) {
        hipStreamSynchronize(bs.s);
        pump_release(p);
        set_error("twa_build_pump: kernel launch failed");
        return TWA_EHIP;
    }
    int rc = factorise(p, bs.s);
    if (rc) {
        pump_release(p);
        return rc;
    }
    *out = p;
    return TWA_OK;
}

TWA_API int twa_build_pump_dense(int64_t N, const double* W_host, twa_pump** out) {
    TWA_API_LOCK();
    using namespace twa;
    if (!out || N < 1 || !W_host) {
        set_error("twa_build_pump_dense: need N >= 1, a matrix and an output pointer");
        return TWA_EINVAL;
    }
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            const double a = W_host[i * N + j], b = W_host[j * N + i];
            if (!std::isfinite(a) || std::fabs(a - b) > 1e-12 * (std::fabs(a) + std::fabs(b))) {
                set_error("twa_build_pump_dense: matrix must be finite and symmetric");
                return TWA_EINVAL;
            }
        }
    *out = nullptr;
    twa_pump* p = new twa_pump();
    p->N = N;
    p->w = NAN;
    p->alpha = NAN;
    hipGetDevice(&p->device);
    if (hipMalloc(&p->W, (size_t)N * N * sizeof(double)) != hipSuccess) {
        delete p;
        set_error("twa_build_pump_dense: device allocation failed");
        return TWA_ENOMEM;
    }
    BuildStream bs;
    if (bs.create("twa_build_pump_dense")) {
        pump_release(p);
        return TWA_EHIP;
    }
    if (hipMemcpyAsync(p->W, W_host, (size_t)N * N * sizeof(double), hipMemcpyHostToDevice, bs.s) != hipSuccess) {
        hipStreamSynchronize(bs.s);
        pump_release(p);
        set_error("twa_build_pump_dense: hipMemcpy failed");
        return TWA_EHIP;
    }
    int rc = factorise(p, bs.s);
    if (rc) {
        pump_release(p);
        return rc;
    }
    *out = p;
    return TWA_OK;
}

TWA_API int twa_build_model_dense(int64_t N, const double* W_host, const double* G_host, const double* Om_host,
                                  twa_pump** out) {
    TWA_API_LOCK();
    using namespace twa;
    if (!out || N < 1 || !W_host || !G_host) {
        set_error("twa_build_model_dense: need N >= 1, two matrices and an output pointer");
        return TWA_EINVAL;
    }
    if (!symmetric_finite(N, W_host) || !symmetric_finite(N, G_host) ||
        (Om_host && !symmetric_finite(N, Om_host))) {
        set_error("twa_build_model_dense: matrices must be finite and symmetric");
        return TWA_EINVAL;
    }
    if (Om_host)
        for (int64_t i = 0; i < N; ++i)
            if (Om_host[i * N + i] != 0.0) {
                set_error("twa_build_model_dense: the exchange matrix must have a zero diagonal");
                return TWA_EINVAL;
            }
    *out = nullptr;
    const size_t bytes = (size_t)N * N * sizeof(double);
    const int64_t n2 = N * N;
    const unsigned nb = (unsigned)((n2 + 255) / 256);
    int rc;
    BuildStream bs;
    if ((rc = bs.create("twa_build_model_dense"))) return rc;
    // the decay matrix itself must be PSD (a physical Lindbladian)
    {
        twa_pump* q = new twa_pump();
        q->N = N;
        q->w = q->alpha = NAN;
        if (hipMalloc(&q->W, bytes) != hipSuccess) {
            delete q;
            set_error("twa_build_model_dense: device allocation failed");
            return TWA_ENOMEM;
        }
        if (hipMemcpyAsync(q->W, G_host, bytes, hipMemcpyHostToDevice, bs.s) != hipSuccess) {
            hipStreamSynchronize(bs.s);
            pump_release(q);
            set_error("twa_build_model_dense: hipMemcpy failed");
            return TWA_EHIP;
        }
        rc = factorise(q, bs.s);
        pump_release(q);
        if (rc == TWA_ENOTPSD) set_error("twa_build_model_dense: decay matrix is not positive semidefinite");
        if (rc) return rc;
    }
    twa_pump* p = new twa_pump();
    p->N = N;
    p->w = NAN;
    p->alpha = NAN;
    hipGetDevice(&p->device);
    double* Wd = nullptr;
    if (hipMalloc(&p->W, bytes) != hipSuccess || hipMalloc(&p->G, bytes) != hipSuccess ||
        hipMalloc(&Wd, bytes) != hipSuccess) {
        hipFree(Wd);
        pump_release(p);
        set_error("twa_build_model_dense: device allocation failed");
        return TWA_ENOMEM;
    }
    if (hipMemcpyAsync(Wd, W_host, bytes, hipMemcpyHostToDevice, bs.s) != hipSuccess ||
        hipMemcpyAsync(p->G, G_host, bytes, hipMemcpyHostToDevice, bs.s) != hipSuccess) {
        hipStreamSynchronize(bs.s);
        hipFree(Wd);
        pump_release(p);
        set_error("twa_build_model_dense: hipMemcpy failed");
        return TWA_EHIP;
    }
    // noise factor of the summed noise: sqrt(W + G); then the drift matrix W - G
    hipLaunchKernelGGL(axpy_kernel, dim3(nb), dim3(256), 0, bs.s, n2, Wd, 1.0, p->G, p->W);
    rc = hipGetLastError() == hipSuccess ? factorise(p, bs.s) : TWA_EHIP;
    if (rc == TWA_OK) {
        hipLaunchKernelGGL(axpy_kernel, dim3(nb), dim3(256), 0, bs.s, n2, Wd, -1.0, p->G, p->W);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(bs.s) != hipSuccess) {
            set_error("twa_build_model_dense: kernel failed");
            rc = TWA_EHIP;
        }
    } else if (rc == TWA_EHIP) {
        set_error("twa_build_model_dense: factorisation of W + G failed");
    }
    hipStreamSynchronize(bs.s);
    hipFree(Wd);
    if (rc == TWA_OK && Om_host) {
        if (hipMalloc(&p->Om, bytes) != hipSuccess) {
            set_error("twa_build_model_dense: device allocation failed");
            rc = TWA_ENOMEM;
        } else if (hipMemcpyAsync(p->Om, Om_host, bytes, hipMemcpyHostToDevice, bs.s) != hipSuccess ||
                   hipStreamSynchronize(bs.s) != hipSuccess) {
            set_error("twa_build_model_dense: hipMemcpy failed");
            rc = TWA_EHIP;
        }
    }
    if (rc) {
        pump_release(p);
        return rc;
    }
    *out = p;
    return TWA_OK;
}

TWA_API int twa_build_pump_toeplitz(int64_t N, double w, double alpha, twa_pump** out) {
    TWA_API_LOCK();
    using namespace twa;
    if (!out || N < 1 || N > toeplitz_max_n(TWA_PREC_FP32) || !std::isfinite(w) || !std::isfinite(alpha) || w < 0 ||
        alpha < 0) {
        set_error("twa_build_pump_toeplitz: need 1 <= N <= 16385, finite w >= 0, finite alpha >= 0 and an output "
                  "pointer");
        return TWA_EINVAL;
    }
    twa_pump* p = new twa_pump();
    p->N = N;
    p->w = w;
    p->alpha = alpha;
    p->lam_min = NAN;
    p->lam_max = toeplitz_spectrum_max(N, w, alpha);
    hipGetDevice(&p->device);
    *out = p;
    return TWA_OK;
}

TWA_API void twa_pump_free(twa_pump* p) {
    TWA_API_LOCK();
    twa::pump_release(p);
}

TWA_API int twa_pump_info(const twa_pump* p, int64_t* N, double* lam_min, double* lam_max) {
    if (!p) {
        twa::set_error("twa_pump_info: NULL handle");
        return TWA_EINVAL;
    }
    if (N) *N = p->N;
    if (lam_min) *lam_min = p->lam_min;
    if (lam_max) *lam_max = p->lam_max;
    return TWA_OK;
}

TWA_API int twa_pump_copy_matrix(const twa_pump* p, int which, double* out_host) {
    TWA_API_LOCK();
    if (!p || !out_host || which < 0 || which > 3 || (which == 2 && !p->G) || (which == 3 && !p->Om)) {
        twa::set_error("twa_pump_copy_matrix: bad arguments (which = 2, 3 need a model handle with G, Omega)");
        return TWA_EINVAL;
    }
    const double* src = which == 0 ? p->W : which == 1 ? p->F : which == 2 ? p->G : p->Om;
    if (!src) {
        twa::set_error("twa_pump_copy_matrix: the handle holds no dense matrices (Toeplitz handle)");
        return TWA_EINVAL;
    }
    twa::BuildStream bs;
    if (bs.create("twa_pump_copy_matrix")) return TWA_EHIP;
    if (hipMemcpyAsync(out_host, src, (size_t)p->N * p->N * sizeof(double), hipMemcpyDeviceToHost, bs.s) !=
            hipSuccess ||
        hipStreamSynchronize(bs.s) != hipSuccess) {
        twa::set_error("twa_pump_copy_matrix: hipMemcpy failed");
        return TWA_EHIP;
    }
    return TWA_OK;
}

}  // extern "C"
