// Toeplitz fast path of the pump of Eq. (2) (not in the paper): on an open
// chain w_ij = c(|i - j|) with c(d) = w / (1 + d)^alpha is a convex
// decreasing sequence, so the Toeplitz matrix embeds in a positive
// semidefinite circulant C of size M = 2^m >= 2N - 2 with first column
// c~_j = c(min(j, M - j)) (Dietrich and Newsam 1997).  With the two spin
// components packed as v = s^x + i s^y:
//   W v      = IDFT(lam * DFT([v; 0]))[:N],
//   pump noise eta = IDFT(sqrt(lam M) * eps)[:N], eps_k complex standard normal,
// whose real and imaginary parts are independent N(0, W) vectors (equal in
// law to the dense path's sqrt(dt) F zeta).  The per-step work drops from
// O(N^2) to O(M log M) per trajectory, and the method becomes an FFT problem
// bound by VALU and LDS, not by the matrix stream.
//
// One workgroup integrates one trajectory over a chunk of steps (both Heun
// stages and the window moments in one launch).  Each thread keeps R complex
// values in registers; a transform is a sequence of Stockham passes (radix R
// first and last, the remainder in between) whose data exchanges go through
// LDS, real and imaginary parts in turn so that M = 32768 FP32 values fit.
// Because the first and last pass both have radix R, a transform reads its
// input and leaves its output in the same natural-strided distribution
// (thread t holds elements t + r T): the pointwise spectral step and the
// per-spin epilogues need no extra exchange.
#include <algorithm>
#include <cmath>
#include <complex>
#include <utility>
#include <vector>

#include "twa_device.h"
#include "twa_internal.h"
#include "twa_run.h"

// Multiply-adds in this file are fused (the library is otherwise built with
// -ffp-contract=off, so that the stage kernels round alike in every variant
// they are inlined into): the transforms are bound by VALU issue and no other
// kernel has to reproduce their rounding.
#pragma clang fp contract(fast)

namespace twa {
namespace {

constexpr uint32_t TAG_CIRCULANT = 3u;   // Philox tag of the circulant normals
constexpr int TOEPLITZ_CHUNK = 256;      // steps per launch

template <typename S>
struct V2;
template <>
struct V2<float> {
    typedef float2 T;
};
template <>
struct V2<double> {
    typedef double2 T;
};

// transform geometry: M = 2^LOGM points, T threads, R = M / T values per thread
template <int LOGM, int LOGR>
struct Plan {
    static constexpr int M = 1 << LOGM, R = 1 << LOGR, T = M / R;
    static constexpr int Q = LOGM / LOGR, REM = LOGM - Q * LOGR;
    static constexpr int NP = Q + (REM ? 1 : 0);
    static constexpr int rad(int p) { return p == 0 ? R : (REM && p == 1) ? (1 << REM) : R; }
    static constexpr int ns(int p) {
        int n = 1;
        for (int i = 0; i < p; ++i) n *= rad(i);
        return n;
    }
    static_assert(Q >= 2, "first and last pass must have radix R");
};

// keeps the scheduler from hoisting the loads of all R slots at once (the
// register arrays already hold 2R values per thread)
#define SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)

constexpr int bitrev(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

// compile-time cos / sin of 2 pi m / n (argument reduced to [-pi, pi], then
// a Taylor series well past double precision): the twiddles of the
// in-register DFTs are literals, not table loads the compiler would keep live
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double reduce(double x) {
    while (x > kPi) x -= 2.0 * kPi;
    while (x < -kPi) x += 2.0 * kPi;
    return x;
}
constexpr double ksin(int m, int n) { return taylor_sin(reduce(2.0 * kPi * m / n)); }
constexpr double kcos(int m, int n) { return taylor_sin(reduce(2.0 * kPi * m / n + 0.5 * kPi)); }

// butterflies of twiddle index MM in the stage of half-size H:
// (a, b) <- (a + w b, a - w b), w = exp(-+2 pi i MM / (2H))
template <typename S, int RAD, int H, int MM, bool INV>
__device__ __forceinline__ void butterflies(S* re, S* im) {
    constexpr S wx = (S)kcos(MM, 2 * H);
    constexpr S wy = (S)(INV ? ksin(MM, 2 * H) : -ksin(MM, 2 * H));
#pragma unroll
    for (int i = 0; i < RAD; i += 2 * H) {
        const int a = i + MM, b = a + H;
        S tr = re[b], ti = im[b];
        if constexpr (MM != 0) {
            tr = re[b] * wx - im[b] * wy;
            ti = re[b] * wy + im[b] * wx;
        }
        re[b] = re[a] - tr;
        im[b] = im[a] - ti;
        re[a] = re[a] + tr;
        im[a] = im[a] + ti;
    }
}

template <typename S, int RAD, int H, bool INV, int... MS>
__device__ __forceinline__ void stage(S* re, S* im, std::integer_sequence<int, MS...>) {
    (butterflies<S, RAD, H, MS, INV>(re, im), ...);
}

template <typename S, int RAD, int H, bool INV>
__device__ __forceinline__ void stages(S* re, S* im) {
    if constexpr (H < RAD) {
        stage<S, RAD, H, INV>(re, im, std::make_integer_sequence<int, H>{});
        stages<S, RAD, 2 * H, INV>(re, im);
    }
}

// in-register RAD-point DFT of re/im[0 .. RAD) in natural order (radix-2
// decimation in time)
template <typename S, int RAD, bool INV>
__device__ __forceinline__ void dft(S* re, S* im) {
    constexpr int LB = ilog2(RAD);
#pragma unroll
    for (int i = 0; i < RAD; ++i) {
        const int j = bitrev(i, LB);
        if (i < j) {
            const S a = re[i], b = im[i];
            re[i] = re[j];
            im[i] = im[j];
            re[j] = a;
            im[j] = b;
        }
    }
    stages<S, RAD, 1, INV>(re, im);
}

// one Stockham pass: positions j = t + g T (g < R / RAD) each take RAD values
// at stride M / RAD (already in registers), twiddle, RAD-point DFT.  The
// twiddle w_M^q is the product of two LDS table entries, w_M^(64 (q >> 6)) and
// w_M^(q & 63).  The thread index is made opaque at the start of the pass (it
// depends on the values just read), so the twiddle addresses are formed here
// and not shared with, or hoisted from, the other passes and transforms.
template <typename S, int M, int T, int R, int RAD, int NS, bool INV>
__device__ __forceinline__ void pass(S (&re)[R], S (&im)[R], int t, const typename V2<S>::T* twh,
                                     const typename V2<S>::T* twl) {
    constexpr int G = R / RAD;
    if constexpr (NS > 1) {
        int tq = t;
        asm volatile("" : "+v"(tq) : "v"(re[0]), "v"(im[0]));
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = tq + g * T;
            const int qs = (j & (NS - 1)) * (M / (NS * RAD));
            // w^r for r = 1 .. RAD-1: a table product at r = 1 and at every
            // fourth r, the others by one more factor w (at most three
            // roundings from a table value), a quarter of the LDS reads
            S w1x = 0, w1y = 0, wx = 0, wy = 0;
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                if (r == 1 || (r & 3) == 0) {
                    const int q = r * qs;
                    const typename V2<S>::T a = twh[q >> 6], b = twl[q & 63];
                    wx = a.x * b.x - a.y * b.y;
                    wy = a.x * b.y + a.y * b.x;
                    if (r == 1) {
                        w1x = wx;
                        w1y = wy;
                    }
                } else {
                    const S nx = wx * w1x - wy * w1y;
                    wy = wx * w1y + wy * w1x;
                    wx = nx;
                }
                const S vy = INV ? -wy : wy;
                const S xr = re[g * RAD + r], xi = im[g * RAD + r];
                re[g * RAD + r] = xr * wx - xi * vy;
                im[g * RAD + r] = xr * vy + xi * wx;
                if ((r & 3) == 3) SCHED_FENCE();
            }
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) dft<S, RAD, INV>(&re[g * RAD], &im[g * RAD]);
}

__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

// LDS exchange between a pass (RAD_A, NS_A) and the next pass (RAD_B): the
// output of slot (g, r) goes to element (j / NS) NS RAD + j % NS + r NS,
// the next pass reads element j' + r' M / RAD_B into slot (g', r').  Element
// e sits at lpad(e) = e + floor(e / 32) (one pad word per 32: stride-32
// stores hit distinct banks).  Both patterns are a per-thread base plus a
// compile-time offset: lpad(base + r NS) = lpad(base) + r NS + floor(r NS / 32)
// because base mod 32 < NS when NS divides 32 and the RAD-group is aligned
// (and exactly when NS is a multiple of 32); likewise for the read stride
// M / RAD_B, a multiple of 32.
template <typename S, int M, int T, int R, int RAD_A, int NS_A, int RAD_B>
__device__ __forceinline__ void exchange_half(S (&v)[R], int t, S* lds) {
    constexpr int GA = R / RAD_A, GB = R / RAD_B, KB = M / RAD_B;
    static_assert(KB % 32 == 0, "read stride must be a multiple of the pad period");
    __syncthreads();
#pragma unroll
    for (int g = 0; g < GA; ++g) {
        const int j = t + g * T;
        S* wb = lds + lpad((j / NS_A) * NS_A * RAD_A + (j % NS_A));
#pragma unroll
        for (int r = 0; r < RAD_A; ++r) wb[r * NS_A + (r * NS_A) / 32] = v[g * RAD_A + r];
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < GB; ++g) {
        const S* rb = lds + lpad(t + g * T);
#pragma unroll
        for (int r = 0; r < RAD_B; ++r) v[g * RAD_B + r] = rb[r * KB + (r * KB) / 32];
    }
}

template <typename S, int M, int T, int R, int RAD_A, int NS_A, int RAD_B>
__device__ __forceinline__ void exchange(S (&re)[R], S (&im)[R], int t, S* lds) {
    exchange_half<S, M, T, R, RAD_A, NS_A, RAD_B>(re, t, lds);
    exchange_half<S, M, T, R, RAD_A, NS_A, RAD_B>(im, t, lds);
}

template <typename S, int LOGM, int LOGR, bool INV, int P>
__device__ __forceinline__ void passes(S (&re)[1 << LOGR], S (&im)[1 << LOGR], int t,
                                       const typename V2<S>::T* twh, const typename V2<S>::T* twl, S* lds) {
    typedef Plan<LOGM, LOGR> PL;
    pass<S, PL::M, PL::T, PL::R, PL::rad(P), PL::ns(P), INV>(re, im, t, twh, twl);
    if constexpr (P + 1 < PL::NP) {
        exchange<S, PL::M, PL::T, PL::R, PL::rad(P), PL::ns(P), PL::rad(P + 1)>(re, im, t, lds);
        passes<S, LOGM, LOGR, INV, P + 1>(re, im, t, twh, twl, lds);
    }
}

// unnormalised DFT (INV = false: exponent -, INV = true: exponent +) of the M
// values held as element t + r T in slot r; the result is held the same way
template <typename S, int LOGM, int LOGR, bool INV>
__device__ __forceinline__ void transform(S (&re)[1 << LOGR], S (&im)[1 << LOGR], int t,
                                          const typename V2<S>::T* twh, const typename V2<S>::T* twl, S* lds) {
    passes<S, LOGM, LOGR, INV, 0>(re, im, t, twh, twl, lds);
}

// the thread index made opaque after a transform: addresses and counters
// derived from it cannot be computed (and their loads issued) before the
// transform is done, which would keep them live across all of its passes
template <typename S, int R>
__device__ __forceinline__ int after(int t, const S (&re)[R], const S (&im)[R]) {
    int q = t;
    asm volatile("" : "+v"(q) : "v"(re[0]), "v"(im[0]), "v"(re[R - 1]), "v"(im[R - 1]));
    return q;
}

// wave sums with ds_swizzle butterflies inside each half-wave (xor 1 .. 16,
// no address registers) and the two halves added in lane 0: a fixed order
template <int PAT>
__device__ __forceinline__ float swz(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), PAT));
}
template <int PAT>
__device__ __forceinline__ double swz(double v) {
    const int2 h = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_ds_swizzle(h.x, PAT),
                                                __builtin_amdgcn_ds_swizzle(h.y, PAT)));
}
__device__ __forceinline__ float lane32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
}
__device__ __forceinline__ double lane32(double v) {
    const int2 h = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(h.x, 32), __builtin_amdgcn_readlane(h.y, 32)));
}
template <typename S>
__device__ __forceinline__ S wave_sum(S v) {
    // swizzle bit mode: and_mask 0x1f, xor_mask m << 10
    v += swz<0x041F>(v);
    v += swz<0x081F>(v);
    v += swz<0x101F>(v);
    v += swz<0x201F>(v);
    v += swz<0x401F>(v);
    return v + lane32(v);   // valid in lane 0
}

// fixed-order workgroup sum of NV values (wave sums, then waves in order)
template <typename S, int T, int NV>
__device__ __forceinline__ void block_sum(S (&v)[NV], S* red) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[wv * NV + q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        S s = red[q];
#pragma unroll
        for (int w = 1; w < T / 64; ++w) s += red[w * NV + q];
        v[q] = s;
    }
}

// per-trajectory planes as raw buffers of N elements: loads past the end
// return 0 and stores past the end are dropped by the hardware, so the
// padding slots (n >= N) of a transform need no branch
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc plane(const void* p, int64_t n_elems, int es) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(n_elems * es), 0x00020000);
}
__device__ __forceinline__ float bld(Rsrc r, int i, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, 0));
}
__device__ __forceinline__ double bld(Rsrc r, int i, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8, 0, 0));
}
__device__ __forceinline__ void bst(Rsrc r, int i, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, i * 4, 0, 0);
}
__device__ __forceinline__ void bst(Rsrc r, int i, double v) {
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) B64;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, v), r, i * 8, 0, 0);
}

template <typename S>
__device__ __forceinline__ void kahan(S& sum, S& comp, S v) {
    const S y = v - comp;
    const S t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

template <typename S, int LOGM, int LOGR>
__global__ __launch_bounds__((1 << LOGM) >> LOGR) void toeplitz_run_kernel(
    int64_t N, int64_t P, int64_t Bp, const typename V2<S>::T* __restrict__ tw,
    const typename V2<S>::T* __restrict__ spec, S c1, S c2, uint32_t k0, uint32_t k1, uint32_t point, int64_t step0,
    int64_t n_steps, int64_t burnin, S* __restrict__ s, S* __restrict__ H, S* __restrict__ mom) {
    typedef Plan<LOGM, LOGR> PL;
    constexpr int M = PL::M, T = PL::T, R = PL::R;
    __shared__ S lds[M + M / 32];
    __shared__ S red[(T / 64) * 3];
    __shared__ typename V2<S>::T twh[M / 64 > 0 ? M / 64 : 1], twl[64];
    const int t = threadIdx.x;
    for (int i = t; i < M / 64; i += T) twh[i] = tw[64 * i];
    for (int i = t; i < 64; i += T) twl[i] = tw[i];
    // (the first block_sum below synchronises before any transform reads them)
    const int64_t k = blockIdx.x;
    const int64_t SP = Bp * P, o = k * P;
    const Rsrc bx = plane(s + o, N, sizeof(S)), by = plane(s + SP + o, N, sizeof(S)),
               bz = plane(s + 2 * SP + o, N, sizeof(S)), bhx = plane(H + o, N, sizeof(S)),
               bhy = plane(H + SP + o, N, sizeof(S));
    S re[R], im[R];
    S xs[3];
    {
        S acc[2] = {0, 0};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            re[r] = bld(bx, t + r * T, S(0));
            im[r] = bld(by, t + r * T, S(0));
            acc[0] += re[r];
            acc[1] += im[r];
            SCHED_FENCE();
        }
        block_sum<S, T, 2>(acc, red);
        xs[0] = acc[0];
        xs[1] = acc[1];
    }
    // Kahan pairs of the window moments live in LDS (thread 0 only), not in
    // registers every thread would carry through the transforms
    __shared__ S kmom[10];
    if (t == 0)
#pragma unroll
        for (int m = 0; m < 10; ++m) kmom[m] = mom[m * Bp + k];
    for (int64_t st = step0; st < step0 + n_steps; ++st) {
        // the thread index made opaque per step: every address below is then
        // recomputed where it is used instead of being kept live (R of each)
        // across the whole step loop
        int tt = t;
        asm volatile("" : "+v"(tt));
        const uint32_t ks = (uint32_t)k, ns = (uint32_t)st;
        S g0, g1;
        {
            const U4 v = philox4x32_10(U4{0u, ks, ns, TAG_COLLECTIVE | (point << 8)}, k0, k1);
            box_muller(v.x, v.y, g0, g1);
        }
        // stage 1: -dt/2 W s - sqrt(dt) eta, through the embedding
        transform<S, LOGM, LOGR, false>(re, im, tt, twh, twl, lds);
        const int t1 = after(tt, re, im);
#pragma unroll
        for (int r = 0; r < R / 2; ++r) {
            const int km = t1 + r * T;   // < M / 2; its partner is km + M / 2 in slot r + R / 2
            const U4 w = philox4x32_10(U4{(uint32_t)km, ks, ns, TAG_CIRCULANT | (point << 8)}, k0, k1);
            S a0, b0, a1, b1;
            box_muller(w.x, w.y, a0, b0);
            box_muller(w.z, w.w, a1, b1);
            const typename V2<S>::T p0 = spec[km], p1 = spec[km + M / 2];
            re[r] = p0.x * re[r] + p0.y * a0;
            im[r] = p0.x * im[r] + p0.y * b0;
            re[r + R / 2] = p1.x * re[r + R / 2] + p1.y * a1;
            im[r + R / 2] = p1.x * im[r + R / 2] + p1.y * b1;
            SCHED_FENCE();
        }
        transform<S, LOGM, LOGR, true>(re, im, tt, twh, twl, lds);
        const int t2 = after(tt, re, im);
        S sd[2] = {0, 0};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // padding slots: z = 0 gives a zero increment, the field store is dropped
            const int n = t2 + r * T;
            const S z = bld(bz, n, S(0));
            const S Hx = re[r] + (c1 * xs[0] + c2 * g0), Hy = im[r] + (c1 * xs[1] + c2 * g1);
            bst(bhx, n, Hx);
            bst(bhy, n, Hy);
            const S dx = z * Hx, dy = z * Hy;
            re[r] = dx;
            im[r] = dy;
            sd[0] += dx;
            sd[1] += dy;
            SCHED_FENCE();
        }
        block_sum<S, T, 2>(sd, red);
        // stage 2: field at the predictor = H + (-dt/2 W Delta) + Gamma dt/2 sum(Delta)
        transform<S, LOGM, LOGR, false>(re, im, tt, twh, twl, lds);
        const int t3 = after(tt, re, im);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const S a = spec[t3 + r * T].x;
            re[r] *= a;
            im[r] *= a;
            SCHED_FENCE();
        }
        transform<S, LOGM, LOGR, true>(re, im, tt, twh, twl, lds);
        const int t4 = after(tt, re, im);
        S acc[3] = {0, 0, 0};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // padding slots load zeros and produce zeros (the next transform's padding)
            const int n = t4 + r * T;
            const S x = bld(bx, n, S(0)), y = bld(by, n, S(0)), z = bld(bz, n, S(0));
            const S Hx = bld(bhx, n, S(0)), Hy = bld(bhy, n, S(0));
            const S dx = z * Hx, dy = z * Hy, dz = -(x * Hx + y * Hy);
            const S px = x + dx, py = y + dy, pz = z + dz;
            const S H2x = Hx + re[r] + c1 * sd[0], H2y = Hy + im[r] + c1 * sd[1];
            const S ex = pz * H2x, ey = pz * H2y, ez = -(px * H2x + py * H2y);
            const S xn = x + S(0.5) * (dx + ex), yn = y + S(0.5) * (dy + ey), zn = z + S(0.5) * (dz + ez);
            bst(bx, n, xn);
            bst(by, n, yn);
            bst(bz, n, zn);
            re[r] = xn;
            im[r] = yn;
            acc[0] += xn;
            acc[1] += yn;
            acc[2] += zn;
            SCHED_FENCE();
        }
        block_sum<S, T, 3>(acc, red);
        xs[0] = acc[0];
        xs[1] = acc[1];
        if (t == 0 && st + 1 > burnin) {
            const S T2 = S(0.25) * (acc[0] * acc[0] + acc[1] * acc[1]);
            const S v[5] = {T2, T2 * acc[2], T2 * T2, acc[2], acc[2] * acc[2]};
#pragma unroll
            for (int m = 0; m < 5; ++m) kahan(kmom[2 * m], kmom[2 * m + 1], v[m]);
        }
    }
    if (t == 0)
#pragma unroll
        for (int m = 0; m < 10; ++m) mom[m * Bp + k] = kmom[m];
}

// host FFT (FP64, radix 2) of the circulant's first column: its eigenvalues
void host_dft(std::vector<std::complex<double>>& a) {
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * M_PI / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t m = 0; m < len / 2; ++m) {
                const std::complex<double> w(std::cos(ang * (double)m), std::sin(ang * (double)m));
                const std::complex<double> u = a[i + m], v = a[i + m + len / 2] * w;
                a[i + m] = u + v;
                a[i + m + len / 2] = u - v;
            }
    }
}

template <typename S, int LOGM, int LOGR>
int launch_t(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const void* tw, const void* spec,
             int64_t step0, int64_t n, int cur, hipStream_t st) {
    typedef typename V2<S>::T S2;
    hipLaunchKernelGGL((toeplitz_run_kernel<S, LOGM, LOGR>), dim3((unsigned)g.B), dim3((1 << LOGM) >> LOGR), 0, st,
                       g.N, g.P, g.Bp, static_cast<const S2*>(tw), static_cast<const S2*>(spec), (S)c.c1, (S)c.c2,
                       c.key0, c.key1, (uint32_t)c.point, step0, n, c.burnin, static_cast<S*>(b.s[cur]),
                       static_cast<S*>(b.Y), static_cast<S*>(b.mom));
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

// (LOGM, LOGR): FP32 keeps R = 32 values per thread (T = M / 32 >= 64),
// FP64 R = 16 (T = M / 16 <= 1024)
template <typename S>
int launch_s(int logm, const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const void* tw,
             const void* spec, int64_t step0, int64_t n, int cur, hipStream_t st) {
    if constexpr (sizeof(S) == 4) {
        switch (logm) {
            case 8: return launch_t<S, 8, 2>(g, b, c, tw, spec, step0, n, cur, st);
            case 9: return launch_t<S, 9, 3>(g, b, c, tw, spec, step0, n, cur, st);
            case 10: return launch_t<S, 10, 4>(g, b, c, tw, spec, step0, n, cur, st);
            case 11: return launch_t<S, 11, 5>(g, b, c, tw, spec, step0, n, cur, st);
            case 12: return launch_t<S, 12, 5>(g, b, c, tw, spec, step0, n, cur, st);
            case 13: return launch_t<S, 13, 5>(g, b, c, tw, spec, step0, n, cur, st);
            case 14: return launch_t<S, 14, 5>(g, b, c, tw, spec, step0, n, cur, st);
            case 15: return launch_t<S, 15, 5>(g, b, c, tw, spec, step0, n, cur, st);
        }
    } else {
        switch (logm) {
            case 8: return launch_t<S, 8, 2>(g, b, c, tw, spec, step0, n, cur, st);
            case 9: return launch_t<S, 9, 3>(g, b, c, tw, spec, step0, n, cur, st);
            case 10: return launch_t<S, 10, 4>(g, b, c, tw, spec, step0, n, cur, st);
            case 11: return launch_t<S, 11, 4>(g, b, c, tw, spec, step0, n, cur, st);
            case 12: return launch_t<S, 12, 4>(g, b, c, tw, spec, step0, n, cur, st);
            case 13: return launch_t<S, 13, 4>(g, b, c, tw, spec, step0, n, cur, st);
            // 512 threads of 32 values: at 1024 threads of 16 each the kernel
            // spilled 87 registers (128 per thread at that size)
            case 14: return launch_t<S, 14, 5>(g, b, c, tw, spec, step0, n, cur, st);
        }
    }
    set_error("Toeplitz path: embedding size out of range");
    return TWA_EINVAL;
}

}  // namespace

double toeplitz_spectrum_max(int64_t N, double w, double alpha) {
    const int64_t M = int64_t(1) << toeplitz_embedding_log2(N);
    std::vector<std::complex<double>> a((size_t)M);
    for (int64_t j = 0; j < M; ++j)
        a[(size_t)j] = std::complex<double>(w / std::pow(1.0 + (double)std::min(j, M - j), alpha), 0.0);
    host_dft(a);
    double m = 0;
    for (const auto& v : a) m = std::max(m, v.real());
    return m;
}

int toeplitz_embedding_log2(int64_t N) {
    int l = 8;
    while ((int64_t(1) << l) < 2 * N - 2) ++l;
    return l;
}

int64_t toeplitz_max_n(int precision) { return precision == TWA_PREC_FP64 ? 8193 : 16385; }

// tables of one run: twiddles w_M^q and the spectral coefficients
// (lam (-dt / 2M), sqrt(lam+) (-sqrt(dt / M))) in the state precision
int toeplitz_tables(const Geometry& g, double w, double alpha, double dt, void** tw, void** spec, hipStream_t st) {
    const int logm = toeplitz_embedding_log2(g.N);
    const int64_t M = int64_t(1) << logm;
    std::vector<std::complex<double>> a((size_t)M);
    for (int64_t j = 0; j < M; ++j) {
        const double d = (double)std::min(j, M - j);
        a[(size_t)j] = std::complex<double>(w / std::pow(1.0 + d, alpha), 0.0);
    }
    host_dft(a);
    double lmax = 0;
    for (int64_t j = 0; j < M; ++j) lmax = std::max(lmax, a[(size_t)j].real());
    const double tol = 8.0 * (double)M * 2.220446049250313e-16 * lmax;
    const bool f64 = g.precision == TWA_PREC_FP64;
    const size_t es = f64 ? 16 : 8;
    std::vector<double> twd((size_t)2 * M), spd((size_t)2 * M);
    for (int64_t q = 0; q < M; ++q) {
        const double ang = 2.0 * M_PI * (double)q / (double)M;
        twd[(size_t)2 * q] = std::cos(ang);
        twd[(size_t)2 * q + 1] = -std::sin(ang);
        const double lam = a[(size_t)q].real();
        spd[(size_t)2 * q] = lam * (-dt / (2.0 * (double)M));
        spd[(size_t)2 * q + 1] = (lam > tol ? std::sqrt(lam) : 0.0) * (-std::sqrt(dt / (double)M));
    }
    if (hipMalloc(tw, (size_t)M * es) != hipSuccess || hipMalloc(spec, (size_t)M * es) != hipSuccess) {
        set_error("Toeplitz path: device allocation failed");
        return TWA_ENOMEM;
    }
    if (f64) {
        if (hipMemcpyAsync(*tw, twd.data(), (size_t)M * es, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(*spec, spd.data(), (size_t)M * es, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("Toeplitz path: hipMemcpy failed");
            return TWA_EHIP;
        }
    } else {
        std::vector<float> t32(twd.begin(), twd.end()), s32(spd.begin(), spd.end());
        if (hipMemcpyAsync(*tw, t32.data(), (size_t)M * es, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(*spec, s32.data(), (size_t)M * es, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("Toeplitz path: hipMemcpy failed");
            return TWA_EHIP;
        }
    }
    return TWA_OK;
}

int launch_toeplitz_run(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, const void* tw,
                        const void* spec, int64_t n_steps, int cur, hipStream_t st) {
    if (g.N > toeplitz_max_n(g.precision)) {
        set_error("Toeplitz path: N exceeds the largest embedding (16385 in FP32, 8193 in FP64)");
        return TWA_EINVAL;
    }
    const int logm = toeplitz_embedding_log2(g.N);
    for (int64_t s0 = 0; s0 < n_steps; s0 += TOEPLITZ_CHUNK) {
        const int64_t n = std::min<int64_t>(TOEPLITZ_CHUNK, n_steps - s0);
        int rc;
        if (g.precision == TWA_PREC_FP64)
            rc = launch_s<double>(logm, g, b, c, tw, spec, s0, n, cur, st);
        else if (g.precision == TWA_PREC_FP32)
            rc = launch_s<float>(logm, g, b, c, tw, spec, s0, n, cur, st);
        else {
            set_error("Toeplitz path: FP64 or FP32 only");
            return TWA_EINVAL;
        }
        if (rc) return rc;
    }
    return TWA_OK;
}

}  // namespace twa
