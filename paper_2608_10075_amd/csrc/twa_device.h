// Device-side building blocks: counter-based noise, number formats of the
// contraction, and the MFMA fragments used by the step kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/twa.h"

namespace twa {

// The constant operand A of a contraction (P rows, K columns) is stored
// stage-blocked: the kt columns of K stage q of all P rows are contiguous,
// row after row, and the stages follow one another.  One LDS stage of MT rows
// is then a single contiguous run of MT * kt elements (whole cache lines),
// where a row-major matrix would give MT runs of kt elements one row pitch
// apart.  kt = K elements per LDS stage of the tile configuration.
__host__ __device__ __forceinline__ int64_t a_index(int64_t i, int64_t j, int64_t P, int64_t kt) {
    return (j / kt) * P * kt + i * kt + (j % kt);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// -> 64-bit multiplies with the published multipliers, the key advanced by
// the published Weyl increments between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // each product as one 64-bit value: one v_mad_u64_u32 instead of a
        // v_mul_hi_u32 and a v_mul_lo_u32 (both quarter rate)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = U4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0};
    }
    return c;
}

// Counter words: (slot, trajectory, step, tag | point << 8).
enum : uint32_t { TAG_PUMP = 0u, TAG_COLLECTIVE = 1u, TAG_INIT = 2u };

// Box-Muller (Box & Muller 1958) on two words.  u1 = ((a >> 8) + 1) 2^-24 in
// (0, 1] and u2 = (b >> 8) 2^-24 are exact in binary32.  Binary32 uses the
// hardware transcendentals: v_log_f32 (log2; ln u1 = ln 2 log2 u1),
// v_sqrt_f32, and v_sin_f32 / v_cos_f32, which take their argument in
// revolutions (sin 2 pi u2 directly, u2 in [0, 1)).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
    const float u1 = (float)((a >> 8) + 1u) * 5.9604644775390625e-08f;
    const float u2 = (float)(b >> 8) * 5.9604644775390625e-08f;
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
    const double u1 = (double)((a >> 8) + 1u) * 5.9604644775390625e-08;
    const double u2 = (double)(b >> 8) * 5.9604644775390625e-08;
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Operand column of component a (0 = x, 1 = y) of trajectory k: x and y of
// 16 consecutive trajectories sit in two adjacent 16-column blocks, so one
// lane of an MFMA output pair holds both components of one (spin, trajectory).
__device__ __forceinline__ int64_t opcol(int64_t k, int a) {
    return 32 * (k >> 4) + 16 * a + (k & 15);
}

// ---------------------------------------------------------------------------
// number formats
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

struct bf16s {
    uint16_t v;
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int PREC>
struct Prec;

template <>
struct Prec<TWA_PREC_FP64> {
    static constexpr int SPLIT = 1;   // operand blocks per value (3: bf16 hi, lo, hi)
    typedef double G;   // contraction operand
    typedef double S;   // state / accumulator
    typedef f64x4 AV;
    // The f64 16x16x4 MFMA returns row (lane/16) + 4 r in register r; feeding
    // A-operand row m with spin 4 (m % 4) + m / 4 makes register r of lane l
    // hold spin 4 (l/16) + r, the layout of the other formats.
    __device__ static __forceinline__ int arow(int m) { return 4 * (m & 3) + (m >> 2); }
    __device__ static __forceinline__ G to_g(S v) { return v; }
    __device__ static __forceinline__ void mma(AV& c, const uint4& a, const uint4& b) {
        const f64x2 fa = __builtin_bit_cast(f64x2, a), fb = __builtin_bit_cast(f64x2, b);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[0], fb[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[1], fb[1], c, 0, 0, 0);
    }
};

template <>
struct Prec<TWA_PREC_FP32> {
    static constexpr int SPLIT = 1;
    // 16x16 MFMA output: register r of lane l holds row 4 (l/16) + r
    __device__ static __forceinline__ int arow(int m) { return m; }
    typedef float G;
    typedef float S;
    typedef f32x4 AV;
    __device__ static __forceinline__ G to_g(S v) { return v; }
    __device__ static __forceinline__ void mma(AV& c, const uint4& a, const uint4& b) {
        const f32x4 fa = __builtin_bit_cast(f32x4, a), fb = __builtin_bit_cast(f32x4, b);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0], fb[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[1], fb[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[2], fb[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[3], fb[3], c, 0, 0, 0);
    }
};

template <>
struct Prec<TWA_PREC_BF16> {
    static constexpr int SPLIT = 1;
    // 16x16 MFMA output: register r of lane l holds row 4 (l/16) + r
    __device__ static __forceinline__ int arow(int m) { return m; }
    typedef bf16s G;
    typedef float S;
    typedef f32x4 AV;
    __device__ static __forceinline__ G to_g(S v) { return G{f32_to_bf16_rne(v)}; }
    __device__ static __forceinline__ void mma(AV& c, const uint4& a, const uint4& b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                    0, 0, 0);
    }
};

template <>
struct Prec<TWA_PREC_FP16> {
    static constexpr int SPLIT = 1;
    // 16x16 MFMA output: register r of lane l holds row 4 (l/16) + r
    __device__ static __forceinline__ int arow(int m) { return m; }
    typedef _Float16 G;
    typedef float S;
    typedef f32x4 AV;
    __device__ static __forceinline__ G to_g(S v) { return (_Float16)v; }
    __device__ static __forceinline__ void mma(AV& c, const uint4& a, const uint4& b) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                   0, 0);
    }
};

// Split BF16: every operand value x is stored as three K blocks (hi, lo, hi)
// with hi = bf16(x), lo = bf16(x - hi), and the pump matrix as (hi, hi, lo),
// so that one BF16 contraction over the tripled K sums Ahi Xhi + Ahi Xlo +
// Alo Xhi; the dropped Alo Xlo and the rounding of lo are O(2^-17) relative.
template <>
struct Prec<TWA_PREC_BF16X3> : Prec<TWA_PREC_BF16> {
    static constexpr int SPLIT = 3;
};

// operand hi / lo parts of a value (for the split form)
__device__ __forceinline__ void bf16_split(float v, uint16_t& hi, uint16_t& lo) {
    hi = f32_to_bf16_rne(v);
    lo = f32_to_bf16_rne(v - bf16_to_f32(hi));
}

// one operand value: p[0], or for the split form (hi, lo, hi) blk elements apart
template <int PREC>
__device__ __forceinline__ void put_op(typename Prec<PREC>::G* p, int64_t blk, typename Prec<PREC>::S v) {
    if constexpr (Prec<PREC>::SPLIT == 3) {
        uint16_t hi, lo;
        bf16_split(v, hi, lo);
        p[0].v = hi;
        p[blk].v = lo;
        p[2 * blk].v = hi;
    } else {
        p[0] = Prec<PREC>::to_g(v);
    }
}

}  // namespace twa
