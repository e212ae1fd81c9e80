// Step kernels of the TWA trajectories (SM Sec. S1, Eq. (S1)) for gfx950.
//
// One stochastic Heun step of Eq. (S1) is two launches of one kernel family:
// a dense channel-mixing contraction on MFMA with the Heun stage fused into
// its epilogue.  With A = [-dt/2 W | -sqrt(dt) F] (W the pump matrix of
// Eq. (2), F its PSD square root) the effective fields of Eq. (S1) over one
// step are
//   stage 1:  H_n  = A [s_n ; zeta]          + (Gamma dt/2) S_n + sqrt(Gamma dt) g
//   stage 2:  H~   = H_n - (Gamma dt/2) S_n + A_left (s~ - s_n) + (Gamma dt/2) S~
// (A_left = -dt/2 W), i.e. the corrector re-uses the stage-1 contraction and
// only contracts the predictor increment, so each step costs three N x N
// operand sweeps per trajectory column (W s, F zeta, W (s~ - s)).  The spin
// update is ds^x = s^z H^x, ds^y = s^z H^y, ds^z = -(s^x H^x + s^y H^y).
//
// The response copies of the two-time correlation (SM Sec. S1, after
// Eq. (S3)) are propagated as tangent-linear copies by the same kernel
// family ("tangent" epilogues) in separate launches that read the primal
// fields of the same step.
//
// Layout: spins of one trajectory contiguous (index k * P + i), trajectory
// operand columns interleaved x/y per 16 trajectories (see opcol).
//
// This header holds the kernel templates; every contraction precision is
// instantiated in a translation unit of its own (twa_step_<precision>.hip),
// and twa_step.hip dispatches to them.
#pragma once

#include <algorithm>
#include <vector>

#include "twa_internal.h"
#include "twa_device.h"

namespace twa {

template <int PREC>
struct GemmArgs {
    typedef typename Prec<PREC>::G G;
    typedef typename Prec<PREC>::S S;
    const G* A;         // P rows, stage-blocked with KB bytes per row and stage (a_index)
    const G* X;         // operand of copy 0
    int64_t ldx;
    int64_t x_copy;     // element offset between copies
    int64_t K;          // contraction length
    int64_t P, Bp, nmt;
    int nnt;            // column tiles
    S c1, c2;
    // primal buffers
    const S* s_cur;
    S* s_next;
    S* dlt;
    S* Y;
    G* Dop;             // stage 1 writes
    int64_t ldd;        // Dop column length (P; SPLIT P in the split form; 2P with coherent exchange)
    int coh;            // coherent exchange: also write the perpendicular blocks (s^y, -s^x) / (D^y, -D^x)
    G* Xnext;           // stage 2 writes (s-part, ld 2P for primal, P for tangents)
    int64_t ldxn;
    const S* part_prim; // primal partial sums read by the epilogue
    S* part_out;        // partial sums written
    const S* g;
    int store_y2;
    S* Sn;              // [2][Bp] collective sums of the input state: stage 1 writes, stage 2 reads
                        // (stage 2 recomputes the predictor increment when dlt is null)
    // tangent buffers (copy 0; copy offsets below)
    const S* t_cur;
    S* t_next;
    S* t_dlt;
    S* tY;
    G* tDop;
    const S* tpart_in;
    int64_t t_state_copy;   // element offset between copies of state-shaped buffers
    int64_t t_y_copy;       // element offset between copies of tY
    int64_t t_part_copy;    // element offset between copies of partial sums
    int64_t t_op_copy;      // element offset between copies of operands
    int64_t* step;          // advanced by stage 2 of the primal (block 0)
    S* Y2out;               // primal stage 2: where the stage-2 field goes (nullptr: in place into Y)
    // store kind: out = in + sign * acc
    const S* Sin;
    S* Sout;
    S store_sign;
    int kq;                 // snapshot kind: K stage at which the second K half starts
    // adjoint kinds (copy cp = objective)
    int64_t N, B;
    const S* Y2in;          // stage-2 contraction output of the primal step
    const S* Qin;           // noise part -sqrt(dt) F zeta of the primal step
    const S* YA;            // d(contraction output)/d(alpha) of the stage
    S* lam;                 // cotangent of the state, [copy][3][Bp][P]
    S* M1;                  // cotangent of the predictor increment
    S* Rb;                  // lam' + cotangent of the predictor state
    double* gacc;           // [copy][2][nmt][Bp] gradient partial sums (w, alpha)
    S inv_w;
    S srccoef[2][5];        // objective coefficients on (T2, T3, T4, Z, ZZ)
    S src_scale;            // 1 / (B * window samples)
    int src_on;             // the state produced by this backward step is observed
};

enum { KIND_PRIMAL = 0, KIND_TANGENT = 1, KIND_STORE = 2, KIND_ADJ2 = 3, KIND_ADJ1 = 4, KIND_SIB = 5,
       KIND_Q_SNAPSHOT = 0x100 };
static_assert(KIND_PRIMAL_WITH_Q == (KIND_PRIMAL | KIND_Q_SNAPSHOT), "kind encoding");

// Semi-implicit midpoint stage (the scheme the paper cites for its
// spin-length-preserving integration): solve s' = s + ((s + s')/2) x b with
// b = (H^y, -H^x, 0) frozen, i.e. (I + [beta]) s' = (I - [beta]) s with
// beta = b/2 and [beta] the matrix of beta x .; the closed-form inverse of
// I + [beta] is (I - [beta] + beta beta^T) / (1 + |beta|^2).  A rotation:
// the spin length is kept exactly (up to rounding).
template <typename S>
__device__ __forceinline__ void midpoint_rotate(S x, S y, S z, S Hx, S Hy, S& ox, S& oy, S& oz) {
    const S bx = S(0.5) * Hy, by = S(-0.5) * Hx;
    // a = s - beta x s, beta x s = (by z, -bx z, bx y - by x)
    const S ax = x - by * z, ay = y + bx * z, az = z - (bx * y - by * x);
    const S bd = bx * ax + by * ay;
    const S inv = S(1) / (S(1) + bx * bx + by * by);
    ox = (ax - by * az + bx * bd) * inv;
    oy = (ay + bx * az + by * bd) * inv;
    oz = (az - (bx * ay - by * ax)) * inv;
}

// The increment s' - s of the same midpoint stage, formed directly rather
// than as a difference of two O(1) vectors (which in binary32 would carry an
// absolute error of the state's rounding, large against an increment of
// O(dt |H|)): s' - s = -2 (I + [beta])^{-1} (beta x s), and with c = beta x s
// (orthogonal to beta) the inverse gives -2 (c - beta x c) / (1 + |beta|^2).
template <typename S>
__device__ __forceinline__ void midpoint_increment(S x, S y, S z, S Hx, S Hy, S& dx, S& dy, S& dz) {
    const S bx = S(0.5) * Hy, by = S(-0.5) * Hx;
    const S cx = by * z, cy = -(bx * z), cz = bx * y - by * x;
    const S f = S(-2) / (S(1) + bx * bx + by * by);
    dx = f * (cx - by * cz);
    dy = f * (cy + bx * cz);
    dz = f * (cz - (bx * cy - by * cx));
}

template <typename S>
__device__ __forceinline__ void ld4(const S* p, S (&v)[4]) {
    if constexpr (sizeof(S) == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
}
template <typename S>
__device__ __forceinline__ void st4(S* p, const S (&v)[4]) {
    if constexpr (sizeof(S) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
    }
}
template <int PREC>
__device__ __forceinline__ void stg4(typename Prec<PREC>::G* p, const typename Prec<PREC>::S (&v)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) p[r] = Prec<PREC>::to_g(v[r]);
}
// coherent exchange: the perpendicular block at row offset off of the x and y
// columns holds (v^y, -v^x)
template <int PREC>
__device__ __forceinline__ void stg4perp(typename Prec<PREC>::G* cx, typename Prec<PREC>::G* cy,
                                         const typename Prec<PREC>::S (&vx)[4], const typename Prec<PREC>::S (&vy)[4]) {
    typename Prec<PREC>::S m[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) m[r] = -vx[r];
    stg4<PREC>(cx, vy);
    stg4<PREC>(cy, m);
}

// Epilogue streams as raw buffers: the descriptor's base is the wave's first
// element of an array (wave-uniform, scalar registers), the lane adds one
// 32-bit byte offset (voff) and the block one uniform byte offset, so every
// stream costs one offset VGPR in total instead of a 64-bit address.  Loads
// take the block offset in the scalar offset field; stores take it in voff
// with a zero scalar offset: with a register scalar offset the compiler puts
// no wait state between a 128-bit store and a VALU write of its data
// registers, and the store then wrote the overwritten value (observed on
// gfx950 in the first dword of a store's data).
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ Rsrc wave_rsrc(const void* base, int64_t bytes) {
    const uint32_t n = bytes >= (int64_t)0xFFFFFFFF ? 0xFFFFFFFFu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n, 0x00020000);
}
// 16 bytes per lane from a raw buffer straight into LDS (lane i to byte 16 i
// of the 1 KB at lds); a MUBUF load, which the compiler counts in vmcnt only
__device__ __forceinline__ void buffer_dma16(Rsrc r, void* lds, uint32_t voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16, voff, 0, 0, 0);
}
template <typename S>
__device__ __forceinline__ void bld4(Rsrc r, uint32_t voff, uint32_t soff, S (&v)[4]) {
    if constexpr (sizeof(S) == 4) {
        const f32x4 t = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
        v[0] = t[0]; v[1] = t[1]; v[2] = t[2]; v[3] = t[3];
    } else {
        const f64x2 t0 = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
        const f64x2 t1 = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0));
        v[0] = t0[0]; v[1] = t0[1]; v[2] = t1[0]; v[3] = t1[1];
    }
}
template <typename S>
__device__ __forceinline__ void bst4(Rsrc r, uint32_t voff, const S (&v)[4]) {
    if constexpr (sizeof(S) == 4) {
        const f32x4 t = {v[0], v[1], v[2], v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t), r, voff, 0, 0);
    } else {
        const f64x2 t0 = {v[0], v[1]}, t1 = {v[2], v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t0), r, voff, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t1), r, voff + 16, 0, 0);
    }
}
// four operand values (contraction type) from state values
template <int PREC>
__device__ __forceinline__ void bstg4(Rsrc r, uint32_t voff, const typename Prec<PREC>::S (&v)[4]) {
    typedef typename Prec<PREC>::G G;
    if constexpr (sizeof(G) == 2) {
        uint16_t h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = __builtin_bit_cast(uint16_t, Prec<PREC>::to_g(v[q]));
        const u32x2 t = {(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16)};
        __builtin_amdgcn_raw_buffer_store_b64(t, r, voff, 0, 0);
    } else {
        typename Prec<PREC>::S g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = Prec<PREC>::to_g(v[q]);
        bst4(r, voff, g);
    }
}
// operand store of a state-like value: one block, or for the split form the
// (hi, lo, hi) blocks blk bytes apart
template <int PREC>
__device__ __forceinline__ void bstg4s(Rsrc r, uint32_t voff, uint32_t blk, const typename Prec<PREC>::S (&v)[4]) {
    if constexpr (Prec<PREC>::SPLIT == 3) {
        uint16_t hi[4], lo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) bf16_split(v[q], hi[q], lo[q]);
        const u32x2 th = {(uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16)};
        const u32x2 tl = {(uint32_t)lo[0] | ((uint32_t)lo[1] << 16), (uint32_t)lo[2] | ((uint32_t)lo[3] << 16)};
        __builtin_amdgcn_raw_buffer_store_b64(th, r, voff, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(tl, r, voff + blk, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(th, r, voff + 2 * blk, 0, 0);
    } else {
        bstg4<PREC>(r, voff, v);
    }
}
// coherent exchange: (v^y, -v^x) into the perpendicular blocks of the x and y
// columns (byte offsets vx_off, vy_off)
template <int PREC>
__device__ __forceinline__ void bstg4perp(Rsrc r, uint32_t vx_off, uint32_t vy_off,
                                          const typename Prec<PREC>::S (&vx)[4],
                                          const typename Prec<PREC>::S (&vy)[4]) {
    typename Prec<PREC>::S m[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = -vx[q];
    bstg4<PREC>(r, vx_off, vy);
    bstg4<PREC>(r, vy_off, m);
}

// operand store of a state-like value: one block, or for the split form the
// (hi, lo, hi) blocks blk elements apart
template <int PREC>
__device__ __forceinline__ void stg4s(typename Prec<PREC>::G* p, int64_t blk, const typename Prec<PREC>::S (&v)[4]) {
    if constexpr (Prec<PREC>::SPLIT == 3) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint16_t hi, lo;
            bf16_split(v[r], hi, lo);
            p[r].v = hi;
            p[blk + r].v = lo;
            p[2 * blk + r].v = hi;
        }
    } else {
        stg4<PREC>(p, v);
    }
}

// ---------------------------------------------------------------------------
// contraction + fused Heun stage
// One output tile (M tile mt of spins, column tile nt, copy cp) of one stage:
// contraction over K on MFMA followed by the fused epilogue of the kind.
template <int PREC, int MT, int NT, int KB, int WMW, int WNW, int NST, int STAGE, int KIND>
__device__ __forceinline__ void stage_tile(const GemmArgs<PREC>& a, const int mt, const int nt, const int cp) {
    // KIND_Q_SNAPSHOT on the predictor kind: also store the part of the
    // contraction that comes from the second K half (the noise columns), by
    // keeping the accumulator at the half-way K stage
    constexpr int KD = KIND & ~KIND_Q_SNAPSHOT;
    constexpr bool QSNAP = (KIND & KIND_Q_SNAPSHOT) != 0;
    static_assert(!QSNAP || (KD == KIND_PRIMAL && STAGE == 1), "snapshot only on the predictor");
    constexpr bool TAN = KD == KIND_TANGENT;
    constexpr bool ADJ = KD == KIND_ADJ2 || KD == KIND_ADJ1;
    constexpr bool TCOPY = TAN || ADJ;     // per-copy collective sums of the copy operand
    typedef typename Prec<PREC>::G G;
    typedef typename Prec<PREC>::S S;
    typedef typename Prec<PREC>::AV AV;
    constexpr int NTHR = 64 * WMW * WNW;
    constexpr int WM = MT / WMW, WN = NT / WNW;
    constexpr int BI = WM / 16, BJ = WN / 16;
    constexpr int PCS = KB / 16;             // 16-byte pieces per row
    constexpr int PA = MT * PCS, PX = NT * PCS;
    constexpr int KT = KB / (int)sizeof(G);
    constexpr int NTRJ = NT / 2;             // trajectories per tile
    static_assert(WM % 16 == 0 && WN % 32 == 0, "wave tile");
    static_assert(KB % 64 == 0, "K stage");

    // NST LDS stages (a ring), each rows [0, MT) of A then [MT, MT + NT) of X,
    // KB bytes per row; inside every 16-row block the 16-byte piece c of row r
    // is stored at piece position c ^ swz(r), which makes the 16-lane fragment
    // reads of one MFMA operand hit distinct LDS banks.  The stages are
    // distinct LDS objects so that the compiler can tell the loads in flight
    // into one stage from the reads of another.
    static_assert(NST >= 2 && NST <= 8, "LDS ring depth");
    constexpr int SB = (MT + NT) * KB;
    __shared__ __attribute__((aligned(1024))) char L0[SB];
    __shared__ __attribute__((aligned(1024))) char L1[SB];
    __shared__ __attribute__((aligned(1024))) char L2[NST > 2 ? SB : 16];
    __shared__ __attribute__((aligned(1024))) char L3[NST > 3 ? SB : 16];
    __shared__ __attribute__((aligned(1024))) char L4[NST > 4 ? SB : 16];
    __shared__ __attribute__((aligned(1024))) char L5[NST > 5 ? SB : 16];
    __shared__ __attribute__((aligned(1024))) char L6[NST > 6 ? SB : 16];
    __shared__ __attribute__((aligned(1024))) char L7[NST > 7 ? SB : 16];
    __shared__ S sS[NTRJ][2];      // primal collective sums of the trajectories of the tile
    __shared__ S sT[NTRJ][2];      // tangent collective sums
    __shared__ S sG[NTRJ][2];      // collective normals
    // cross-wave partial sums: [wave row][trajectory][4 channels] in the
    // epilogue, [thread group][trajectory][5 channels] for the collective sums
    constexpr int NG = NTHR / NTRJ;            // thread groups of the collective sums
    static_assert(NTHR % NTRJ == 0, "thread groups");
    __shared__ S red[WMW > NG ? WMW : NG][NTRJ][5];
    __shared__ S sSrc[NTRJ][3];    // adjoint: observation source of each trajectory

    const int64_t m0 = (int64_t)mt * MT, n0 = (int64_t)nt * NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WMW, wn = wave / WMW;
    const int wm0 = wm * WM, wn0 = wn * WN;
    const int64_t P = a.P, Bp = a.Bp, nmt = a.nmt;
    const int64_t k0t = n0 / 2;    // first trajectory of the tile

    // ---- main loop: acc[i][col] = sum_k A[m0+i][k] X[n0+col][k]
    AV acc[BI][BJ];
    AV accW[QSNAP ? BI : 1][QSNAP ? BJ : 1];   // accumulator at K stage kq (snapshot kind)
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) acc[i][j] = AV{0, 0, 0, 0};

    // A is stage-blocked: row r of K stage q at byte (q P + r) KB; X columns
    // are row-major with a pitch of ldx elements
    const char* Ag = reinterpret_cast<const char*>(a.A) + m0 * KB;
    const char* Xg = reinterpret_cast<const char*>(a.X + cp * a.x_copy + n0 * a.ldx);
    const int64_t ldx_b = a.ldx * (int64_t)sizeof(G);
    const int nk = (int)(a.K / KT);
    // Direct memory -> LDS loads (buffer_load_dwordx4 ... lds): one wave
    // instruction moves 64 x 16 bytes into 1 KB of LDS, lane i to offset 16 i,
    // so each lane fetches the piece that belongs at its slot.  The buffer
    // form, not global_load_lds: the compiler takes a FLAT-encoded load into
    // LDS for a possible out-of-order LDS access and then waits for every
    // fragment read before the first MFMA of a stage (lgkmcnt(0)); with the
    // buffer form it waits for each read only where its MFMA needs it.  A
    // stage's descriptors span exactly this tile's rows of that stage (A:
    // MT rows of KB bytes; X: NT rows at a pitch of ldx elements), so no
    // load can leave them; the offsets fit 32 bits for any A that fits in
    // device memory.
    constexpr int RPC = 1024 / KB;                 // rows per 1 KB chunk
    constexpr int NCH = (MT + NT) / RPC;           // chunks per stage
    constexpr int NWV = NTHR / 64;
    constexpr int CPW = (NCH + NWV - 1) / NWV;     // chunks per wave per stage (at most)
    constexpr int CPWMIN = NCH / NWV;              // (at least)
    static_assert(MT % RPC == 0 && (MT + NT) % RPC == 0, "chunking");
    // (gfx950 serves a 16-byte LDS read in four passes of 16 lanes over 64
    // four-byte banks; these swizzles make every pass of the fragment reads
    // conflict free, for the FP64 row order as well)
    auto swz = [](int r16) {
        return PREC == TWA_PREC_FP64 ? (r16 ^ (r16 >> 2)) % PCS : (PCS >= 16 ? r16 : r16 >> 1) % PCS;
    };
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    uint32_t voff[CPW];           // lane's byte offset in its chunk's operand rows of one stage
    bool srcA[CPW];               // chunk j holds rows of A (else of X); wave-uniform
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int q = wv + j * NWV < NCH ? wv + j * NWV : 0;
        const int row = q * RPC + lane / PCS;
        const int pc = (lane % PCS) ^ swz(row & 15);
        srcA[j] = q * RPC < MT;
        voff[j] = row < MT ? (uint32_t)(row * KB + pc * 16) : (uint32_t)((row - MT) * ldx_b + pc * 16);
    }
    const int64_t astage_b = P * KB;   // bytes between K stages of A
    const int64_t a_stage_bytes = (int64_t)MT * KB;               // this tile's A rows of one stage
    const int64_t x_stage_bytes = (int64_t)(NT - 1) * ldx_b + KB; // its X rows of one stage
#define TWA_DMA(KT_, BUF_)                                                                              \
    do {                                                                                                \
        const Rsrc ra_ = wave_rsrc(Ag + (int64_t)(KT_) * astage_b, a_stage_bytes);                      \
        const Rsrc rx_ = wave_rsrc(Xg + (int64_t)(KT_) * KB, x_stage_bytes);                            \
        _Pragma("unroll") for (int j = 0; j < CPW; ++j) if (CPW == CPWMIN || wv + j * NWV < NCH)        \
            buffer_dma16(srcA[j] ? ra_ : rx_, (BUF_) + (wv + j * NWV) * 1024, voff[j]);                  \
    } while (0)

    // fragment read offsets of this lane (row within a 16-row block, swizzle)
    const int ra = Prec<PREC>::arow(lane & 15), rx = lane & 15;
    const int offA = (wm0 + ra) * KB, offX = (MT + wn0 + rx) * KB;
    const int swA = swz(ra), swX = swz(rx), grp = lane >> 4;
#define TWA_BUF(I_) ((I_) == 0 ? L0 : (I_) == 1 ? L1 : (I_) == 2 ? L2 : (I_) == 3 ? L3 : \
                     (I_) == 4 ? L4 : (I_) == 5 ? L5 : (I_) == 6 ? L6 : L7)
    // vmcnt-only wait (expcnt and lgkmcnt left at their maxima), gfx9 encoding
#define TWA_WAIT_VM(N_) __builtin_amdgcn_s_waitcnt(((N_) & 15) | (((N_) >> 4) << 14) | (7 << 4) | (15 << 8))

#define TWA_COMPUTE(BUF_)                                                                               \
    do {                                                                                                \
        _Pragma("unroll") for (int seg = 0; seg < KB / 64; ++seg) {                                     \
            uint4 af[BI], xf[BJ];                                                                       \
            const int c_ = seg * 4 + grp;                                                               \
            _Pragma("unroll") for (int i = 0; i < BI; ++i) af[i] = *reinterpret_cast<const uint4*>(     \
                (BUF_) + offA + 16 * i * KB + ((c_ ^ swA) << 4));                                       \
            _Pragma("unroll") for (int j = 0; j < BJ; ++j) xf[j] = *reinterpret_cast<const uint4*>(     \
                (BUF_) + offX + 16 * j * KB + ((c_ ^ swX) << 4));                                       \
            _Pragma("unroll") for (int i = 0; i < BI; ++i)                                              \
                _Pragma("unroll") for (int j = 0; j < BJ; ++j) Prec<PREC>::mma(acc[i][j], af[i], xf[j]); \
        }                                                                                               \
    } while (0)
#define TWA_BUF(I_) ((I_) == 0 ? L0 : (I_) == 1 ? L1 : (I_) == 2 ? L2 : (I_) == 3 ? L3 : \
                     (I_) == 4 ? L4 : (I_) == 5 ? L5 : (I_) == 6 ? L6 : L7)
    // vmcnt-only wait (expcnt and lgkmcnt left at their maxima), gfx9 encoding
#define TWA_WAIT_VM(N_) __builtin_amdgcn_s_waitcnt(((N_) & 15) | (((N_) >> 4) << 14) | (7 << 4) | (15 << 8))


    // ---- collective sums of this tile's trajectories: thread group g of
    // trajectory kl adds the partial sums of the M tiles
    // q in [g nmt / NG, (g+1) nmt / NG) in order, then the groups are added in
    // order (a fixed summation order: the result does not depend on timing).
    // Channels: 0, 1 primal x, y; 2, 3 copy x, y; 4 primal z.
    if constexpr (KD != KIND_STORE) {
        constexpr int NCHAN = KD == KIND_ADJ1 ? 5 : TCOPY ? 4 : 2;
        {
            const int kl = tid % NTRJ, gq = tid / NTRJ;
            const int64_t k = k0t + kl;
            const int64_t q0 = nmt * gq / NG, q1 = nmt * (gq + 1) / NG;
            const S* pp = a.part_prim;
            const S* tp = TCOPY ? a.tpart_in + cp * a.t_part_copy : nullptr;
            S v[5] = {0, 0, 0, 0, 0};
#pragma unroll 4
            for (int64_t q = q0; q < q1; ++q) {
                v[0] += pp[(0 * nmt + q) * Bp + k];
                v[1] += pp[(1 * nmt + q) * Bp + k];
                if constexpr (TCOPY) {
                    v[2] += tp[(0 * nmt + q) * Bp + k];
                    v[3] += tp[(1 * nmt + q) * Bp + k];
                }
                if constexpr (KD == KIND_ADJ1) v[4] += pp[(2 * nmt + q) * Bp + k];
            }
#pragma unroll
            for (int c = 0; c < NCHAN; ++c) red[gq][kl][c] = v[c];
        }
        __syncthreads();
        for (int t = tid; t < NTRJ; t += NTHR) {
            const int64_t k = k0t + t;
            S v[5];
#pragma unroll
            for (int c = 0; c < NCHAN; ++c) {
                v[c] = red[0][t][c];
                for (int g2 = 1; g2 < NG; ++g2) v[c] += red[g2][t][c];
            }
            const S sx = v[0], sy = v[1];
            sS[t][0] = sx;
            sS[t][1] = sy;
            if constexpr (KD == KIND_PRIMAL || KD == KIND_SIB) {
                if (a.Sn) {
                    if constexpr (STAGE == 1) {
                        if (mt == 0) {
                            a.Sn[k] = sx;
                            a.Sn[Bp + k] = sy;
                        }
                    } else if (a.dlt == nullptr || KD == KIND_SIB) {
                        // sums of the step's input state, for the predictor increment
                        sT[t][0] = a.Sn[k];
                        sT[t][1] = a.Sn[Bp + k];
                    }
                }
            }
            sG[t][0] = a.g[k];
            sG[t][1] = a.g[Bp + k];
            if constexpr (TCOPY) {
                sT[t][0] = v[2];
                sT[t][1] = v[3];
            }
            if constexpr (KD == KIND_ADJ1) {
                // derivative of the observed moments (T2, T3, T4, Z, ZZ) of this
                // trajectory's state with respect to any one spin component
                const S sz = v[4];
                S ox = 0, oy = 0, oz = 0;
                if (a.src_on && k < a.B) {
                    const S T2 = S(0.25) * (sx * sx + sy * sy);
                    const S* cf = a.srccoef[cp];
                    const S gt = S(0.5) * cf[0] + S(0.5) * cf[1] * sz + cf[2] * T2;
                    ox = a.src_scale * gt * sx;
                    oy = a.src_scale * gt * sy;
                    oz = a.src_scale * (cf[1] * T2 + cf[3] + S(2) * cf[4] * sz);
                }
                sSrc[t][0] = ox;
                sSrc[t][1] = oy;
                sSrc[t][2] = oz;
            }
        }
        __syncthreads();   // the sums are visible to every wave; red is free again
    }
    // prologue: stages 0 .. NST-2 in flight
#pragma unroll
    for (int u = 0; u < NST - 1; ++u)
        if (u < nk) TWA_DMA(u, TWA_BUF(u));
    for (int kt0 = 0; kt0 < nk; kt0 += NST) {
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int kt = kt0 + u;
            if (kt < nk) {
                // stage kt has landed once at most the later stages are pending
                // (waves that load fewer chunks per stage wait conservatively)
                if (nk - 1 - kt >= NST - 2) TWA_WAIT_VM((NST - 2) * CPWMIN);
                else TWA_WAIT_VM(0);
                // Barrier without a memory fence: a fence would wait for every
                // load still in flight into the later stages.  What it has to
                // order is covered explicitly: this wave's loads into stage kt
                // completed (vmcnt above), and its reads of the stage the next
                // load overwrites were consumed by MFMAs before this point.
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                if (kt + NST - 1 < nk) TWA_DMA(kt + NST - 1, TWA_BUF((u + NST - 1) % NST));
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (QSNAP) {
                    if (kt == a.kq) {
#pragma unroll
                        for (int i = 0; i < BI; ++i)
#pragma unroll
                            for (int j = 0; j < BJ; ++j) accW[i][j] = acc[i][j];
                    }
                }
                TWA_COMPUTE(TWA_BUF(u));
            }
        }
    }
#undef TWA_DMA
#undef TWA_COMPUTE
#undef TWA_BUF
#undef TWA_WAIT_VM

    // ---- epilogue: fused Heun stage on (spin i, trajectory k)
    const S c1 = a.c1, c2 = a.c2;
    const int64_t SP = Bp * P;   // plane size
    // The primal kinds load the state (and, in the corrector, the predictor
    // field) of the next (p, bi) block before the current block is computed
    // and stored, so one block of loads is always in flight behind the stores
    // instead of every block waiting out a full memory round trip.
    // Their addresses: a buffer descriptor per array plane based at the wave's
    // first element, one lane byte offset per layout (state planes [k][P],
    // operand columns of the next contraction) and a uniform byte offset per
    // block (p, bi).
    constexpr bool PF = KD == KIND_PRIMAL || KD == KIND_SIB;
    constexpr int NPF = STAGE == 2 ? 5 : 3;
    constexpr int NBLK = (BJ / 2) * BI;
    const int wvu = __builtin_amdgcn_readfirstlane(wave);
    const int64_t wm0u = (int64_t)(wvu % WMW) * WM, kw0 = k0t + (int64_t)(wvu / WMW) * (WN / 2);
    const int64_t eb_s = kw0 * P + m0 + wm0u;                 // wave base in a state plane
    const int64_t rem_s = (SP - eb_s) * (int64_t)sizeof(S);
    const uint32_t lane_s = (uint32_t)(((lane & 15) * P + 4 * (lane >> 4)) * (int64_t)sizeof(S));
    auto so_s = [&](const int p, const int bi) { return (uint32_t)((16 * p * P + 16 * bi) * (int64_t)sizeof(S)); };
    auto plane = [&](const S* arr, const int c) { return wave_rsrc(arr + c * SP + eb_s, rem_s); };
    // operand columns: trajectory kw0 + 16 p + (lane & 15) has columns
    // opcol(k, c) = 32 (kw0 / 16 + p) + 16 c + (lane & 15), rows m0 + wm0u + ...
    auto op_rsrc = [&](const G* arr, const int64_t ld) {
        const int64_t eb = 32 * (kw0 >> 4) * ld + m0 + wm0u;
        return wave_rsrc(arr + eb, (2 * Bp * ld - eb) * (int64_t)sizeof(G));
    };
    auto op_lane = [&](const int64_t ld) {
        return (uint32_t)(((lane & 15) * ld + 4 * (lane >> 4)) * (int64_t)sizeof(G));
    };
    auto so_op = [&](const int64_t ld, const int p, const int c, const int bi, const int64_t row) {
        return (uint32_t)(((32 * p + 16 * c) * ld + row + 16 * bi) * (int64_t)sizeof(G));
    };
    const uint32_t blk_b = (uint32_t)(P * (int64_t)sizeof(G));   // split (hi, lo, hi) block stride
    Rsrc rs[3], ry[2], rop;
    uint32_t ld_d = 0, ld_x = 0;
    if constexpr (PF) {
#pragma unroll
        for (int c = 0; c < 3; ++c) rs[c] = plane(a.s_cur, c);
#pragma unroll
        for (int c = 0; c < 2; ++c) ry[c] = plane(a.Y, c);
        if constexpr (STAGE == 1) {
            rop = op_rsrc(a.Dop, a.ldd);
            ld_d = op_lane(a.ldd);
        } else {
            rop = op_rsrc(a.Xnext, a.ldxn);
            ld_x = op_lane(a.ldxn);
        }
    }
    S pfn[NPF][4];
    auto pf_load = [&](const int p, const int bi) {
        const uint32_t so = so_s(p, bi);
        bld4(rs[0], lane_s, so, pfn[0]);
        bld4(rs[1], lane_s, so, pfn[1]);
        bld4(rs[2], lane_s, so, pfn[2]);
        if constexpr (NPF == 5) {
            bld4(ry[0], lane_s, so, pfn[3]);
            bld4(ry[1], lane_s, so, pfn[4]);
        }
    };
    if constexpr (PF) pf_load(0, 0);
#pragma unroll
    for (int p = 0; p < BJ / 2; ++p) {
        const int kl = wn0 / 2 + 16 * p + (lane & 15);
        const int64_t k = k0t + kl;
        const S Sx = sS[kl][0], Sy = sS[kl][1];
        const S hx0 = c1 * Sx + c2 * sG[kl][0];
        const S hy0 = c1 * Sy + c2 * sG[kl][1];
        S ps0 = 0, ps1 = 0, ps2 = 0, ps3 = 0;
#pragma unroll
        for (int bi = 0; bi < BI; ++bi) {
            const int64_t i0 = m0 + wm0 + 16 * bi + 4 * (lane >> 4);
            const int64_t off = k * P + i0;
            S x[4], y[4], z[4], fyx[4], fyy[4], fdx[4], fdy[4], fdz[4];
            if constexpr (PF) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    x[r] = pfn[0][r];
                    y[r] = pfn[1][r];
                    z[r] = pfn[2][r];
                    if constexpr (NPF == 5) {
                        fyx[r] = pfn[3][r];
                        fyy[r] = pfn[4][r];
                    }
                }
                // the stored predictor increment (when kept) is read before the
                // next block's loads are issued, so that its wait does not
                // include them
                if constexpr (KD == KIND_PRIMAL && STAGE == 2) {
                    if (a.dlt) {
                        bld4(plane(a.dlt, 0), lane_s, so_s(p, bi), fdx);
                        bld4(plane(a.dlt, 1), lane_s, so_s(p, bi), fdy);
                        bld4(plane(a.dlt, 2), lane_s, so_s(p, bi), fdz);
                    }
                }
                if (p * BI + bi + 1 < NBLK) pf_load((p * BI + bi + 1) / BI, (p * BI + bi + 1) % BI);
            } else if constexpr (KD != KIND_STORE) {
                ld4(a.s_cur + off, x);
                ld4(a.s_cur + SP + off, y);
                ld4(a.s_cur + 2 * SP + off, z);
            }
            if constexpr (KD == KIND_PRIMAL && STAGE == 1) {
                S dx[4], dy[4], dz[4], yx[4], yy[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S ax = acc[bi][2 * p][r], ay = acc[bi][2 * p + 1][r];
                    const S Hx = ax + hx0, Hy = ay + hy0;
                    dx[r] = z[r] * Hx;
                    dy[r] = z[r] * Hy;
                    dz[r] = -(x[r] * Hx + y[r] * Hy);
                    yx[r] = ax;
                    yy[r] = ay;
                    ps0 += x[r] + dx[r];
                    ps1 += y[r] + dy[r];
                    ps2 += z[r] + dz[r];
                }
                if (a.dlt) {
                    bst4(plane(a.dlt, 0), lane_s + so_s(p, bi), dx);
                    bst4(plane(a.dlt, 1), lane_s + so_s(p, bi), dy);
                    bst4(plane(a.dlt, 2), lane_s + so_s(p, bi), dz);
                }
                bst4(ry[0], lane_s + so_s(p, bi), yx);
                bst4(ry[1], lane_s + so_s(p, bi), yy);
                bstg4s<PREC>(rop, ld_d + so_op(a.ldd, p, 0, bi, 0), blk_b, dx);
                bstg4s<PREC>(rop, ld_d + so_op(a.ldd, p, 1, bi, 0), blk_b, dy);
                if (a.coh)
                    bstg4perp<PREC>(rop, ld_d + so_op(a.ldd, p, 0, bi, P), ld_d + so_op(a.ldd, p, 1, bi, P), dx, dy);
                if constexpr (QSNAP) {
                    S qx[4], qy[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        qx[r] = acc[bi][2 * p][r] - accW[bi][2 * p][r];
                        qy[r] = acc[bi][2 * p + 1][r] - accW[bi][2 * p + 1][r];
                    }
                    bst4(plane(a.Sout, 0), lane_s + so_s(p, bi), qx);
                    bst4(plane(a.Sout, 1), lane_s + so_s(p, bi), qy);
                }
            } else if constexpr (KD == KIND_SIB && STAGE == 1) {
                // predictor: the midpoint rule with the field at s_n; its
                // increment D (the corrector's operand) formed directly
                S dx[4], dy[4], yx[4], yy[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S ax = acc[bi][2 * p][r], ay = acc[bi][2 * p + 1][r];
                    S dz;
                    midpoint_increment(x[r], y[r], z[r], ax + hx0, ay + hy0, dx[r], dy[r], dz);
                    yx[r] = ax;
                    yy[r] = ay;
                    ps0 += x[r] + dx[r];
                    ps1 += y[r] + dy[r];
                    ps2 += z[r] + dz;
                }
                bst4(ry[0], lane_s + so_s(p, bi), yx);
                bst4(ry[1], lane_s + so_s(p, bi), yy);
                bstg4s<PREC>(rop, ld_d + so_op(a.ldd, p, 0, bi, 0), blk_b, dx);
                bstg4s<PREC>(rop, ld_d + so_op(a.ldd, p, 1, bi, 0), blk_b, dy);
                if (a.coh)
                    bstg4perp<PREC>(rop, ld_d + so_op(a.ldd, p, 0, bi, P), ld_d + so_op(a.ldd, p, 1, bi, P), dx, dy);
            } else if constexpr (KD == KIND_SIB && STAGE == 2) {
                // corrector: the midpoint rule from s_n with the field at the
                // midpoint m = s_n + D/2: contraction Y1 + A_left D / 2, sums (S_n + S~)/2
                S nx[4], ny[4], nz[4];
                const S (&yx)[4] = fyx;
                const S (&yy)[4] = fyy;
                const S hxm = c1 * (S(0.5) * (sT[kl][0] + Sx)) + c2 * sG[kl][0];
                const S hym = c1 * (S(0.5) * (sT[kl][1] + Sy)) + c2 * sG[kl][1];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S Hx = (yx[r] + S(0.5) * acc[bi][2 * p][r]) + hxm;
                    const S Hy = (yy[r] + S(0.5) * acc[bi][2 * p + 1][r]) + hym;
                    midpoint_rotate(x[r], y[r], z[r], Hx, Hy, nx[r], ny[r], nz[r]);
                    ps0 += nx[r];
                    ps1 += ny[r];
                    ps2 += nz[r];
                }
                bst4(plane(a.s_next, 0), lane_s + so_s(p, bi), nx);
                bst4(plane(a.s_next, 1), lane_s + so_s(p, bi), ny);
                bst4(plane(a.s_next, 2), lane_s + so_s(p, bi), nz);
                bstg4s<PREC>(rop, ld_x + so_op(a.ldxn, p, 0, bi, 0), blk_b, nx);
                bstg4s<PREC>(rop, ld_x + so_op(a.ldxn, p, 1, bi, 0), blk_b, ny);
                if (a.coh)
                    bstg4perp<PREC>(rop, ld_x + so_op(a.ldxn, p, 0, bi, 2 * P), ld_x + so_op(a.ldxn, p, 1, bi, 2 * P),
                                    nx, ny);
            } else if constexpr (KD == KIND_PRIMAL && STAGE == 2) {
                S dx[4], dy[4], dz[4], yx[4], yy[4], nx[4], ny[4], nz[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    yx[r] = fyx[r];
                    yy[r] = fyy[r];
                }
                if (a.dlt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        dx[r] = fdx[r];
                        dy[r] = fdy[r];
                        dz[r] = fdz[r];
                    }
                } else {
                    // the predictor increment, recomputed exactly as the predictor
                    // stage formed it (same operands, same operation order)
                    const S hxn = c1 * sT[kl][0] + c2 * sG[kl][0];
                    const S hyn = c1 * sT[kl][1] + c2 * sG[kl][1];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const S Hx = yx[r] + hxn, Hy = yy[r] + hyn;
                        dx[r] = z[r] * Hx;
                        dy[r] = z[r] * Hy;
                        dz[r] = -(x[r] * Hx + y[r] * Hy);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S ax = yx[r] + acc[bi][2 * p][r], ay = yy[r] + acc[bi][2 * p + 1][r];
                    const S Hx = ax + hx0, Hy = ay + hy0;
                    const S px = x[r] + dx[r], py = y[r] + dy[r], pz = z[r] + dz[r];
                    const S ex = pz * Hx, ey = pz * Hy, ez = -(px * Hx + py * Hy);
                    nx[r] = x[r] + S(0.5) * (dx[r] + ex);
                    ny[r] = y[r] + S(0.5) * (dy[r] + ey);
                    nz[r] = z[r] + S(0.5) * (dz[r] + ez);
                    yx[r] = ax;
                    yy[r] = ay;
                    ps0 += nx[r];
                    ps1 += ny[r];
                    ps2 += nz[r];
                }
                bst4(plane(a.s_next, 0), lane_s + so_s(p, bi), nx);
                bst4(plane(a.s_next, 1), lane_s + so_s(p, bi), ny);
                bst4(plane(a.s_next, 2), lane_s + so_s(p, bi), nz);
                if (a.store_y2) {
                    const S* yo = a.Y2out ? a.Y2out : a.Y;
                    bst4(plane(yo, 0), lane_s + so_s(p, bi), yx);
                    bst4(plane(yo, 1), lane_s + so_s(p, bi), yy);
                }
                bstg4s<PREC>(rop, ld_x + so_op(a.ldxn, p, 0, bi, 0), blk_b, nx);
                bstg4s<PREC>(rop, ld_x + so_op(a.ldxn, p, 1, bi, 0), blk_b, ny);
                if (a.coh)
                    bstg4perp<PREC>(rop, ld_x + so_op(a.ldxn, p, 0, bi, 2 * P), ld_x + so_op(a.ldxn, p, 1, bi, 2 * P),
                                    nx, ny);
            } else if constexpr (KD == KIND_TANGENT && STAGE == 1) {
                const S tSx = sT[kl][0], tSy = sT[kl][1];
                const S* tc = a.t_cur + cp * a.t_state_copy;
                S u[4], v[4], w[4], yx[4], yy[4], ex[4], ey[4], ez[4], ax4[4], ay4[4];
                ld4(tc + off, u);
                ld4(tc + SP + off, v);
                ld4(tc + 2 * SP + off, w);
                ld4(a.Y + off, yx);
                ld4(a.Y + SP + off, yy);
                // parameter tangent in w: the field's own derivative
                // dH/dw = Y/w - Q/(2w) (W linear, F square-root homogeneous in w)
                S sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
                if (a.Qin) {
                    S qx[4], qy[4];
                    ld4(a.Qin + off, qx);
                    ld4(a.Qin + SP + off, qy);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        sx[r] = yx[r] * a.inv_w - S(0.5) * a.inv_w * qx[r];
                        sy[r] = yy[r] * a.inv_w - S(0.5) * a.inv_w * qy[r];
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S Hx = yx[r] + hx0, Hy = yy[r] + hy0;
                    const S ax = acc[bi][2 * p][r], ay = acc[bi][2 * p + 1][r];
                    const S dHx = ax + c1 * tSx + sx[r], dHy = ay + c1 * tSy + sy[r];
                    ex[r] = w[r] * Hx + z[r] * dHx;
                    ey[r] = w[r] * Hy + z[r] * dHy;
                    ez[r] = -(u[r] * Hx + x[r] * dHx + v[r] * Hy + y[r] * dHy);
                    ax4[r] = ax;
                    ay4[r] = ay;
                    ps0 += u[r] + ex[r];
                    ps1 += v[r] + ey[r];
                    ps2 += w[r] + ez[r];
                }
                S* td = a.t_dlt + cp * a.t_state_copy;
                S* ty = a.tY + cp * a.t_y_copy;
                st4(td + off, ex);
                st4(td + SP + off, ey);
                st4(td + 2 * SP + off, ez);
                st4(ty + off, ax4);
                st4(ty + SP + off, ay4);
                G* tdo = a.tDop + cp * a.t_op_copy;
                constexpr int SPLT = Prec<PREC>::SPLIT;
                stg4s<PREC>(tdo + opcol(k, 0) * P * SPLT + i0, P, ex);
                stg4s<PREC>(tdo + opcol(k, 1) * P * SPLT + i0, P, ey);
            } else if constexpr (KD == KIND_STORE) {
                S ox[4], oy[4];
                if (a.Sin) {
                    ld4(a.Sin + off, ox);
                    ld4(a.Sin + SP + off, oy);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) ox[r] = oy[r] = S(0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ox[r] += a.store_sign * acc[bi][2 * p][r];
                    oy[r] += a.store_sign * acc[bi][2 * p + 1][r];
                }
                st4(a.Sout + off, ox);
                st4(a.Sout + SP + off, oy);
            } else if constexpr (KD == KIND_ADJ2) {
                // reverse of the corrector: lam' -> (mu1, R = lam' + cotangent of s~, nu1)
                const int64_t co = cp * a.t_state_copy;
                S lx[4], ly[4], lz[4], dx[4], dy[4], dz[4], y2x[4], y2y[4], qx[4], qy[4], ax_[4], ay_[4];
                ld4(a.lam + co + off, lx);
                ld4(a.lam + co + SP + off, ly);
                ld4(a.lam + co + 2 * SP + off, lz);
                ld4(a.dlt + off, dx);
                ld4(a.dlt + SP + off, dy);
                ld4(a.dlt + 2 * SP + off, dz);
                ld4(a.Y2in + off, y2x);
                ld4(a.Y2in + SP + off, y2y);
                ld4(a.Qin + off, qx);
                ld4(a.Qin + SP + off, qy);
                ld4(a.YA + off, ax_);
                ld4(a.YA + SP + off, ay_);
                const S tSx = sT[kl][0], tSy = sT[kl][1];
                S m1x[4], m1y[4], m1z[4], rx[4], ry[4], rz[4], n1x[4], n1y[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S px = x[r] + dx[r], py = y[r] + dy[r], pz = z[r] + dz[r];
                    const S Hx = y2x[r] + hx0, Hy = y2y[r] + hy0;
                    const S ux = S(0.5) * lx[r], uy = S(0.5) * ly[r], uz = S(0.5) * lz[r];
                    const S n2x = ux * pz - uz * px, n2y = uy * pz - uz * py;
                    const S tx = -uz * Hx + c1 * tSx + acc[bi][2 * p][r];
                    const S ty = -uz * Hy + c1 * tSy + acc[bi][2 * p + 1][r];
                    const S tz = ux * Hx + uy * Hy;
                    m1x[r] = ux + tx;
                    m1y[r] = uy + ty;
                    m1z[r] = uz + tz;
                    rx[r] = lx[r] + tx;
                    ry[r] = ly[r] + ty;
                    rz[r] = lz[r] + tz;
                    n1x[r] = m1x[r] * z[r] - m1z[r] * x[r];
                    n1y[r] = m1y[r] * z[r] - m1z[r] * y[r];
                    ps0 += n1x[r];
                    ps1 += n1y[r];
                    ps2 += n2x * (y2x[r] * a.inv_w - S(0.5) * a.inv_w * qx[r]) +
                           n2y * (y2y[r] * a.inv_w - S(0.5) * a.inv_w * qy[r]);
                    ps3 += n2x * ax_[r] + n2y * ay_[r];
                }
                st4(a.M1 + co + off, m1x);
                st4(a.M1 + co + SP + off, m1y);
                st4(a.M1 + co + 2 * SP + off, m1z);
                st4(a.Rb + co + off, rx);
                st4(a.Rb + co + SP + off, ry);
                st4(a.Rb + co + 2 * SP + off, rz);
                G* no = a.Xnext + cp * a.t_op_copy;
                stg4s<PREC>(no + opcol(k, 0) * a.ldxn + i0, P, n1x);
                stg4s<PREC>(no + opcol(k, 1) * a.ldxn + i0, P, n1y);
            } else if constexpr (KD == KIND_ADJ1) {
                // reverse of the predictor: (mu1, R) -> lam of the step's input state
                const int64_t co = cp * a.t_state_copy;
                S mx[4], my[4], mz[4], rx[4], ry[4], rz[4], y1x[4], y1y[4], qx[4], qy[4], ax_[4], ay_[4];
                ld4(a.M1 + co + off, mx);
                ld4(a.M1 + co + SP + off, my);
                ld4(a.M1 + co + 2 * SP + off, mz);
                ld4(a.Rb + co + off, rx);
                ld4(a.Rb + co + SP + off, ry);
                ld4(a.Rb + co + 2 * SP + off, rz);
                ld4(a.Y + off, y1x);
                ld4(a.Y + SP + off, y1y);
                ld4(a.Qin + off, qx);
                ld4(a.Qin + SP + off, qy);
                ld4(a.YA + off, ax_);
                ld4(a.YA + SP + off, ay_);
                const S tSx = sT[kl][0], tSy = sT[kl][1];
                const S ox = sSrc[kl][0], oy = sSrc[kl][1], oz = sSrc[kl][2];
                S nlx[4], nly[4], nlz[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S Hx = y1x[r] + hx0, Hy = y1y[r] + hy0;
                    const S msk = (i0 + r < a.N) ? S(1) : S(0);
                    nlx[r] = rx[r] - mz[r] * Hx + c1 * tSx + acc[bi][2 * p][r] + msk * ox;
                    nly[r] = ry[r] - mz[r] * Hy + c1 * tSy + acc[bi][2 * p + 1][r] + msk * oy;
                    nlz[r] = rz[r] + mx[r] * Hx + my[r] * Hy + msk * oz;
                    const S n1x = mx[r] * z[r] - mz[r] * x[r], n1y = my[r] * z[r] - mz[r] * y[r];
                    ps2 += n1x * (y1x[r] * a.inv_w - S(0.5) * a.inv_w * qx[r]) +
                           n1y * (y1y[r] * a.inv_w - S(0.5) * a.inv_w * qy[r]);
                    ps3 += n1x * ax_[r] + n1y * ay_[r];
                }
                st4(a.lam + co + off, nlx);
                st4(a.lam + co + SP + off, nly);
                st4(a.lam + co + 2 * SP + off, nlz);
            } else {  // KIND_TANGENT && STAGE == 2
                const S tSx = sT[kl][0], tSy = sT[kl][1];
                const S* tc = a.t_cur + cp * a.t_state_copy;
                const S* td = a.t_dlt + cp * a.t_state_copy;
                const S* ty = a.tY + cp * a.t_y_copy;
                S dx[4], dy[4], dz[4], yx[4], yy[4];
                ld4(a.dlt + off, dx);
                ld4(a.dlt + SP + off, dy);
                ld4(a.dlt + 2 * SP + off, dz);
                ld4(a.Y + off, yx);
                ld4(a.Y + SP + off, yy);
                S u[4], v[4], w[4], du[4], dv[4], dw[4], tyx[4], tyy[4], nu[4], nv[4], nw[4];
                ld4(tc + off, u);
                ld4(tc + SP + off, v);
                ld4(tc + 2 * SP + off, w);
                ld4(td + off, du);
                ld4(td + SP + off, dv);
                ld4(td + 2 * SP + off, dw);
                ld4(ty + off, tyx);
                ld4(ty + SP + off, tyy);
                // parameter tangent in w: dH~/dw = Y2/w - Q/(2w), Y2 the corrector's field
                S sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0};
                if (a.Qin) {
                    S qx[4], qy[4];
                    ld4(a.Qin + off, qx);
                    ld4(a.Qin + SP + off, qy);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        sx[r] = yx[r] * a.inv_w - S(0.5) * a.inv_w * qx[r];
                        sy[r] = yy[r] * a.inv_w - S(0.5) * a.inv_w * qy[r];
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S px = x[r] + dx[r], py = y[r] + dy[r], pz = z[r] + dz[r];
                    const S Hx = yx[r] + hx0, Hy = yy[r] + hy0;
                    const S pu = u[r] + du[r], pv = v[r] + dv[r], pw = w[r] + dw[r];
                    const S dHx = tyx[r] + acc[bi][2 * p][r] + c1 * tSx + sx[r];
                    const S dHy = tyy[r] + acc[bi][2 * p + 1][r] + c1 * tSy + sy[r];
                    const S ex = pw * Hx + pz * dHx;
                    const S ey = pw * Hy + pz * dHy;
                    const S ez = -(pu * Hx + px * dHx + pv * Hy + py * dHy);
                    nu[r] = u[r] + S(0.5) * (du[r] + ex);
                    nv[r] = v[r] + S(0.5) * (dv[r] + ey);
                    nw[r] = w[r] + S(0.5) * (dw[r] + ez);
                    ps0 += nu[r];
                    ps1 += nv[r];
                    ps2 += nw[r];
                }
                S* tn = a.t_next + cp * a.t_state_copy;
                st4(tn + off, nu);
                st4(tn + SP + off, nv);
                st4(tn + 2 * SP + off, nw);
                G* txo = a.Xnext + cp * a.t_op_copy;
                stg4s<PREC>(txo + opcol(k, 0) * a.ldxn + i0, P, nu);
                stg4s<PREC>(txo + opcol(k, 1) * a.ldxn + i0, P, nv);
            }
            // the partial sums are formed inside their block (an empty asm pins
            // each sum in a register here): sunk to the end of the group, they
            // kept every block's state live and spilled it
            if constexpr (PF) {
                asm volatile("" : "+v"(ps0), "+v"(ps1), "+v"(ps2));
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // partial spin sums of the new values: lanes sharing a trajectory,
        // then waves along M, in a fixed order
        ps0 += __shfl_xor(ps0, 16);
        ps1 += __shfl_xor(ps1, 16);
        ps2 += __shfl_xor(ps2, 16);
        ps3 += __shfl_xor(ps3, 16);
        ps0 += __shfl_xor(ps0, 32);
        ps1 += __shfl_xor(ps1, 32);
        ps2 += __shfl_xor(ps2, 32);
        ps3 += __shfl_xor(ps3, 32);
        if (lane < 16) {
            red[wm][kl][0] = ps0;
            red[wm][kl][1] = ps1;
            red[wm][kl][2] = ps2;
            red[wm][kl][3] = ps3;
        }
    }
    if constexpr (KD != KIND_STORE) {
        __syncthreads();
        if constexpr (KD == KIND_PRIMAL || KD == KIND_SIB || KD == KIND_TANGENT || KD == KIND_ADJ2) {
            // ADJ2: channels 0, 1 are the spin sums of nu1 (its z channel is zero)
            S* po = a.part_out + (TCOPY ? cp * a.t_part_copy : 0);
            for (int t = tid; t < 3 * NTRJ; t += NTHR) {
                const int c = t / NTRJ, kl = t % NTRJ;
                S sum = 0;
                if (KD != KIND_ADJ2 || c < 2) {
#pragma unroll
                    for (int q = 0; q < WMW; ++q) sum += red[q][kl][c];
                }
                po[((int64_t)c * nmt + mt) * Bp + k0t + kl] = sum;
            }
        }
        if constexpr (ADJ) {
            // gradient channels 2 (w) and 3 (alpha), accumulated over steps in FP64;
            // each (copy, M tile, trajectory) slot belongs to one workgroup
            for (int t = tid; t < 2 * NTRJ; t += NTHR) {
                const int c = t / NTRJ, kl = t % NTRJ;
                S sum = 0;
#pragma unroll
                for (int q = 0; q < WMW; ++q) sum += red[q][kl][2 + c];
                double* gp = a.gacc + (((int64_t)cp * 2 + c) * nmt + mt) * Bp + k0t + kl;
                *gp += (double)sum;
            }
        }
    }
}

// One launch = one stage of one ensemble.  XCD-aware tile order: workgroups
// are dispatched round-robin over the 8 XCDs, so workgroup b runs on XCD b % 8.
// Each XCD is given a contiguous range of tiles ordered M-tile-major, so the
// workgroups resident on one XCD share the same rows of A (and walk K
// together) in that XCD's L2.
template <int PREC, int MT, int NT, int KB, int WMW, int WNW, int NST, int STAGE, int KIND>
__global__ __launch_bounds__(64 * WMW * WNW) void heun_stage_kernel(GemmArgs<PREC> a) {
    const int nnt = a.nnt;            // column tiles
    const int T = (int)gridDim.x;     // total tiles = nmt * nnt
    const int q = T / 8, r = T % 8;
    const int b = (int)blockIdx.x, x = b % 8, j = b / 8;
    const int L = x * q + (x < r ? x : r) + j;
    stage_tile<PREC, MT, NT, KB, WMW, WNW, NST, STAGE, KIND>(a, L / nnt, L % nnt, (int)blockIdx.z);
    if constexpr ((KIND == KIND_PRIMAL || KIND == KIND_SIB) && STAGE == 2) {
        if (blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x == 0) a.step[0] += 1;
    }
}

// Grouped persistent launch: the stage of many independent ensembles (the
// points of a parameter scan), each with its own arguments, over one tile
// list (point, M tile, column tile, copy) ordered longest-first; workgroup b
// takes tiles b, b + grid, b + 2 grid, ...
template <int PREC, int MT, int NT, int KB, int WMW, int WNW, int NST, int STAGE, int KIND>
__global__ __launch_bounds__(64 * WMW * WNW) void heun_stage_grouped(const GemmArgs<PREC>* __restrict__ args,
                                                                     const int4* __restrict__ tiles, int ntiles,
                                                                     int64_t* step) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tt = tiles[t];
        __syncthreads();   // LDS of the previous tile is free
        stage_tile<PREC, MT, NT, KB, WMW, WNW, NST, STAGE, KIND>(args[tt.x], tt.y, tt.z, tt.w);
    }
    if constexpr ((KIND == KIND_PRIMAL || KIND == KIND_SIB) && STAGE == 2) {
        if (blockIdx.x == 0 && threadIdx.x == 0) step[0] += 1;
    }
}

template <int PREC, int CFG>
struct CfgT;
#define TWA_CFG(ID, MT_, NT_, KB_, WM_, WN_, NST_)  \
    template <int PREC>                             \
    struct CfgT<PREC, ID> {                         \
        static constexpr int MT = MT_, NT = NT_, KB = KB_, WMW = WM_, WNW = WN_, NST = NST_; \
    };
TWA_CFG(0, 16, 32, 64, 1, 1, 2)
TWA_CFG(1, 64, 64, 64, 2, 2, 4)
TWA_CFG(2, 128, 128, 128, 2, 2, 4)
TWA_CFG(3, 128, 128, 64, 2, 2, 8)
TWA_CFG(4, 256, 128, 64, 4, 1, 6)
TWA_CFG(5, 128, 256, 64, 2, 2, 6)
TWA_CFG(6, 256, 128, 64, 4, 2, 4)
TWA_CFG(7, 320, 256, 128, 4, 2, 2)
TWA_CFG(8, 320, 256, 64, 4, 2, 4)

// The contraction loop reaches a stage's X rows by 32-bit byte offsets from
// the stage's base: NT - 1 rows at a pitch of ldx elements plus one K stage
// must stay within 4 GiB (beyond it the buffer loads would return zeros).
template <int PREC>
static bool x_offsets_fit(int64_t ldx, int nt, int kbytes) {
    return (int64_t)(nt - 1) * ldx * (int64_t)sizeof(typename Prec<PREC>::G) + kbytes <= (int64_t)0xFFFFFFFF;
}

template <int PREC, int CFG, int STAGE, int KIND>
static int launch_kernel(const GemmArgs<PREC>& a, int64_t P, int64_t C2, int ncopy, hipStream_t st) {
    typedef CfgT<PREC, CFG> C;
    if (!x_offsets_fit<PREC>(a.ldx, C::NT, C::KB)) {
        set_error("operand pitch too large for the contraction's 32-bit offsets");
        return TWA_EINVAL;
    }
    GemmArgs<PREC> aa = a;
    aa.nnt = (int)(C2 / C::NT);
    dim3 grid((unsigned)((P / C::MT) * (C2 / C::NT)), 1u, (unsigned)ncopy);
    dim3 block(64 * C::WMW * C::WNW);
    hipLaunchKernelGGL((heun_stage_kernel<PREC, C::MT, C::NT, C::KB, C::WMW, C::WNW, C::NST, STAGE, KIND>), grid,
                       block, 0, st, aa);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <int PREC, int CFG>
static int dispatch_kind(const GemmArgs<PREC>& a, int stage, int kind, int64_t P, int64_t C2, int ncopy,
                         hipStream_t st) {
    if constexpr (Prec<PREC>::SPLIT == 3) {
        // the split form runs the forward step and the forward-mode tangent
        // (with the predictor that keeps its noise part)
        if (kind == KIND_PRIMAL)
            return stage == 1 ? launch_kernel<PREC, CFG, 1, KIND_PRIMAL>(a, P, C2, ncopy, st)
                              : launch_kernel<PREC, CFG, 2, KIND_PRIMAL>(a, P, C2, ncopy, st);
        if (kind == KIND_SIB)
            return stage == 1 ? launch_kernel<PREC, CFG, 1, KIND_SIB>(a, P, C2, ncopy, st)
                              : launch_kernel<PREC, CFG, 2, KIND_SIB>(a, P, C2, ncopy, st);
        if (kind == KIND_TANGENT)
            return stage == 1 ? launch_kernel<PREC, CFG, 1, KIND_TANGENT>(a, P, C2, ncopy, st)
                              : launch_kernel<PREC, CFG, 2, KIND_TANGENT>(a, P, C2, ncopy, st);
        if (kind == (KIND_PRIMAL | KIND_Q_SNAPSHOT) && stage == 1)
            return launch_kernel<PREC, CFG, 1, KIND_PRIMAL | KIND_Q_SNAPSHOT>(a, P, C2, ncopy, st);
        if (kind == KIND_STORE && stage == 1) return launch_kernel<PREC, CFG, 1, KIND_STORE>(a, P, C2, ncopy, st);
        if (kind == KIND_ADJ1 && stage == 1) return launch_kernel<PREC, CFG, 1, KIND_ADJ1>(a, P, C2, ncopy, st);
        if (kind == KIND_ADJ2 && stage == 2) return launch_kernel<PREC, CFG, 2, KIND_ADJ2>(a, P, C2, ncopy, st);
        set_error("split BF16: unsupported step kind");
        return TWA_EINVAL;
    } else {
        if (stage == 1) {
            switch (kind) {
                case KIND_PRIMAL: return launch_kernel<PREC, CFG, 1, KIND_PRIMAL>(a, P, C2, ncopy, st);
                case KIND_SIB: return launch_kernel<PREC, CFG, 1, KIND_SIB>(a, P, C2, ncopy, st);
                case KIND_TANGENT: return launch_kernel<PREC, CFG, 1, KIND_TANGENT>(a, P, C2, ncopy, st);
                case KIND_STORE: return launch_kernel<PREC, CFG, 1, KIND_STORE>(a, P, C2, ncopy, st);
                case KIND_PRIMAL | KIND_Q_SNAPSHOT:
                    return launch_kernel<PREC, CFG, 1, KIND_PRIMAL | KIND_Q_SNAPSHOT>(a, P, C2, ncopy, st);
                case KIND_ADJ1: return launch_kernel<PREC, CFG, 1, KIND_ADJ1>(a, P, C2, ncopy, st);
            }
        } else {
            switch (kind) {
                case KIND_PRIMAL: return launch_kernel<PREC, CFG, 2, KIND_PRIMAL>(a, P, C2, ncopy, st);
                case KIND_SIB: return launch_kernel<PREC, CFG, 2, KIND_SIB>(a, P, C2, ncopy, st);
                case KIND_TANGENT: return launch_kernel<PREC, CFG, 2, KIND_TANGENT>(a, P, C2, ncopy, st);
                case KIND_ADJ2: return launch_kernel<PREC, CFG, 2, KIND_ADJ2>(a, P, C2, ncopy, st);
            }
        }
    }
    set_error("unsupported (stage, kind) combination");
    return TWA_EINVAL;
}

template <int PREC>
static int dispatch_cfg(const GemmArgs<PREC>& a, int cfg, int stage, int kind, int64_t P, int64_t C2, int ncopy,
                        hipStream_t st) {
    switch (cfg) {
        case 0: return dispatch_kind<PREC, 0>(a, stage, kind, P, C2, ncopy, st);
        case 1: return dispatch_kind<PREC, 1>(a, stage, kind, P, C2, ncopy, st);
        case 2: return dispatch_kind<PREC, 2>(a, stage, kind, P, C2, ncopy, st);
        case 3: return dispatch_kind<PREC, 3>(a, stage, kind, P, C2, ncopy, st);
    }
    if constexpr (PREC != TWA_PREC_FP64) {
        switch (cfg) {
            case 4: return dispatch_kind<PREC, 4>(a, stage, kind, P, C2, ncopy, st);
            case 5: return dispatch_kind<PREC, 5>(a, stage, kind, P, C2, ncopy, st);
            case 6: return dispatch_kind<PREC, 6>(a, stage, kind, P, C2, ncopy, st);
            case 7: return dispatch_kind<PREC, 7>(a, stage, kind, P, C2, ncopy, st);
            case 8: return dispatch_kind<PREC, 8>(a, stage, kind, P, C2, ncopy, st);
        }
    }
    set_error("unknown tile configuration");
    return TWA_EINVAL;
}

// arguments of a forward-run contraction launch (primal or response copies)
template <int PREC>
static GemmArgs<PREC> make_args(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage,
                                bool tangent, int cur, bool store_y2, bool keep_dlt) {
    typedef typename Prec<PREC>::G G;
    typedef typename Prec<PREC>::S S;
    GemmArgs<PREC> a{};
    const int64_t P = g.P, Bp = g.Bp;
    constexpr int SPL = Prec<PREC>::SPLIT;   // K blocks per value (split form: hi, lo, hi)
    const int64_t CK = g.coh ? 1 : 0;         // coherent exchange: one more K block (s_perp, D_perp)
    a.A = static_cast<const G*>(b.A);
    a.ldd = (1 + CK) * P * SPL;
    a.coh = g.coh;
    a.P = P;
    a.Bp = Bp;
    a.nmt = g.nmt;
    a.N = g.N;
    a.B = g.B;
    a.c1 = (S)c.c1;
    a.c2 = (S)c.c2;
    a.s_cur = static_cast<const S*>(b.s[cur]);
    a.s_next = static_cast<S*>(b.s[1 - cur]);
    a.dlt = (tangent || keep_dlt) ? static_cast<S*>(b.dlt) : nullptr;
    a.Sn = static_cast<S*>(b.Sn);
    a.Y = static_cast<S*>(b.Y);
    a.Dop = static_cast<G*>(b.Dop);
    a.g = static_cast<const S*>(b.g);
    a.store_y2 = store_y2 ? 1 : 0;
    a.step = b.step;
    a.t_state_copy = 3 * Bp * P;
    a.t_y_copy = 2 * Bp * P;
    a.t_part_copy = 3 * g.nmt * Bp;
    a.t_op_copy = g.C2 * P * SPL;
    if (!tangent) {
        if (stage == 1) {
            a.X = static_cast<const G*>(b.Xop);
            a.ldx = (2 + CK) * P * SPL;
            a.K = (2 + CK) * P * SPL;
            a.part_prim = static_cast<const S*>(b.part[0]);
            a.part_out = static_cast<S*>(b.part[1]);
        } else {
            if (CK) a.A = static_cast<const G*>(b.A2);   // corrector: [-dt/2 W | dt Omega] against (D, D_perp)
            a.X = static_cast<const G*>(b.Dop);
            a.ldx = (1 + CK) * P * SPL;
            a.K = (1 + CK) * P * SPL;
            a.part_prim = static_cast<const S*>(b.part[1]);
            a.part_out = static_cast<S*>(b.part[0]);
            a.Xnext = static_cast<G*>(b.Xop);
            a.ldxn = (2 + CK) * P * SPL;
        }
    } else {
        a.t_cur = static_cast<const S*>(b.ts[cur]);
        a.t_next = static_cast<S*>(b.ts[1 - cur]);
        a.t_dlt = static_cast<S*>(b.tdlt);
        a.tY = static_cast<S*>(b.tY);
        a.tDop = static_cast<G*>(b.tDop);
        a.x_copy = g.C2 * P * SPL;
        a.K = P * SPL;
        a.ldx = P * SPL;
        if (stage == 1) {
            a.X = static_cast<const G*>(b.tXop);
            a.part_prim = static_cast<const S*>(b.part[0]);
            a.tpart_in = static_cast<const S*>(b.tpart[0]);
            a.part_out = static_cast<S*>(b.tpart[1]);
        } else {
            a.X = static_cast<const G*>(b.tDop);
            a.part_prim = static_cast<const S*>(b.part[1]);
            a.tpart_in = static_cast<const S*>(b.tpart[1]);
            a.part_out = static_cast<S*>(b.tpart[0]);
            a.Xnext = static_cast<G*>(b.tXop);
            a.ldxn = P * SPL;
        }
    }
    return a;
}

template <int PREC>
int launch_gemm_p(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage,
                         bool tangent, int cur, bool store_y2, bool keep_dlt, hipStream_t st) {
    const GemmArgs<PREC> a = make_args<PREC>(g, b, c, stage, tangent, cur, store_y2, keep_dlt);
    const int kind = tangent ? KIND_TANGENT : g.integrator == TWA_INT_SIB ? KIND_SIB : KIND_PRIMAL;
    return dispatch_cfg<PREC>(a, g.cfg, stage, kind, g.P, g.C2, tangent ? 2 : 1,
                              st);
}

// generic launch from a type-erased call description (adjoint driver)
template <int PREC>
int launch_call_p(const Geometry& g, const GemmCall& c, hipStream_t st) {
    typedef typename Prec<PREC>::G G;
    typedef typename Prec<PREC>::S S;
    GemmArgs<PREC> a{};
    a.A = static_cast<const G*>(c.A);
    a.X = static_cast<const G*>(c.X);
    a.ldx = c.ldx;
    a.x_copy = c.x_copy;
    a.K = c.K;
    a.P = g.P;
    a.Bp = g.Bp;
    a.nmt = g.nmt;
    a.N = g.N;
    a.B = g.B;
    a.c1 = (S)c.c1;
    a.c2 = (S)c.c2;
    a.s_cur = static_cast<const S*>(c.s_cur);
    a.s_next = static_cast<S*>(c.s_next);
    a.dlt = static_cast<S*>(c.dlt);
    a.Y = static_cast<S*>(c.Y);
    a.Y2out = static_cast<S*>(c.Y2out);
    a.Dop = static_cast<G*>(c.Dop);
    a.ldd = g.P * Prec<PREC>::SPLIT;
    a.coh = 0;
    a.Xnext = static_cast<G*>(c.Xnext);
    a.ldxn = c.ldxn;
    a.part_prim = static_cast<const S*>(c.part_prim);
    a.part_out = static_cast<S*>(c.part_out);
    a.g = static_cast<const S*>(c.g);
    a.store_y2 = c.store_y2;
    a.tpart_in = static_cast<const S*>(c.tpart_in);
    a.t_cur = static_cast<const S*>(c.t_cur);
    a.t_next = static_cast<S*>(c.t_next);
    a.t_dlt = static_cast<S*>(c.t_dlt);
    a.tY = static_cast<S*>(c.tY);
    a.tDop = static_cast<G*>(c.tDop);
    a.t_state_copy = 3 * g.Bp * g.P;
    a.t_y_copy = 2 * g.Bp * g.P;
    a.t_part_copy = 3 * g.nmt * g.Bp;
    a.t_op_copy = g.C2 * g.P * Prec<PREC>::SPLIT;
    a.step = c.step;
    a.Sin = static_cast<const S*>(c.Sin);
    a.Sout = static_cast<S*>(c.Sout);
    a.store_sign = (S)c.store_sign;
    a.kq = (int)(g.P * Prec<PREC>::SPLIT / g.kt);   // K stage where the noise columns start
    a.Y2in = static_cast<const S*>(c.Y2in);
    a.Qin = static_cast<const S*>(c.Qin);
    a.YA = static_cast<const S*>(c.YA);
    a.lam = static_cast<S*>(c.lam);
    a.M1 = static_cast<S*>(c.M1);
    a.Rb = static_cast<S*>(c.Rb);
    a.gacc = c.gacc;
    a.inv_w = (S)c.inv_w;
    for (int q = 0; q < 2; ++q)
        for (int m = 0; m < 5; ++m) a.srccoef[q][m] = (S)c.srccoef[q][m];
    a.src_scale = (S)c.src_scale;
    a.src_on = c.src_on;
    return dispatch_cfg<PREC>(a, g.cfg, c.stage, c.kind, g.P, g.C2, c.ncopy, st);
}

// ---------------------------------------------------------------------------
// grouped persistent launches of many ensembles (batched parameter scan)
template <int PREC, int CFG, int STAGE, int KIND>
static int grouped_launch_k(const GroupedPlan& pl, int cur, int variant, hipStream_t st) {
    typedef CfgT<PREC, CFG> C;
    const int tl = variant == GV_TANGENT ? 1 : 0;
    hipLaunchKernelGGL((heun_stage_grouped<PREC, C::MT, C::NT, C::KB, C::WMW, C::WNW, C::NST, STAGE, KIND>),
                       dim3((unsigned)pl.grid[tl]), dim3(64 * C::WMW * C::WNW), 0, st,
                       static_cast<const GemmArgs<PREC>*>(pl.d_args[variant][STAGE - 1][cur]), pl.d_tiles[tl],
                       pl.ntiles[tl], pl.step);
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <int PREC, int CFG, int STAGE>
static int grouped_launch_t(const GroupedPlan& pl, int cur, int variant, hipStream_t st) {
    if (variant == GV_TANGENT) return grouped_launch_k<PREC, CFG, STAGE, KIND_TANGENT>(pl, cur, variant, st);
    return pl.integrator == TWA_INT_SIB ? grouped_launch_k<PREC, CFG, STAGE, KIND_SIB>(pl, cur, variant, st)
                                        : grouped_launch_k<PREC, CFG, STAGE, KIND_PRIMAL>(pl, cur, variant, st);
}

template <int PREC, int CFG>
static int grouped_occupancy() {
    typedef CfgT<PREC, CFG> C;
    int nb = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, heun_stage_grouped<PREC, C::MT, C::NT, C::KB, C::WMW, C::WNW, C::NST, 1, KIND_PRIMAL>,
        64 * C::WMW * C::WNW, 0);
    return nb > 0 ? nb : 1;
}

template <int PREC, int CFG>
static int grouped_dispatch(const GroupedPlan& pl, int stage, int cur, int variant, hipStream_t st) {
    return stage == 1 ? grouped_launch_t<PREC, CFG, 1>(pl, cur, variant, st)
                      : grouped_launch_t<PREC, CFG, 2>(pl, cur, variant, st);
}

// XCD-aware order of a tile list: within every full round of `grid` tiles,
// XCD x (workgroups w with w % 8 == x) gets a contiguous block of the list
inline void xcd_permute(std::vector<int4>& tiles, int grid) {
    const int ntl = (int)tiles.size();
    if (grid % 8 != 0) return;
    std::vector<int4> perm(tiles);
    const int per = grid / 8;
    for (int r0 = 0; r0 + grid <= ntl; r0 += grid)
        for (int w = 0; w < grid; ++w) perm[(size_t)(r0 + w)] = tiles[(size_t)(r0 + (w % 8) * per + w / 8)];
    tiles.swap(perm);
}

template <int PREC>
int grouped_prepare_p(const std::vector<Geometry>& gs, const std::vector<EnsembleBuffers>& bs,
                             const std::vector<StepConsts>& cs, int64_t* step, bool tangents, GroupedPlan& pl,
                             hipStream_t st) {
    const int np = (int)gs.size();
    const int cfg = gs[0].cfg;
    const TileCfg& tc = tile_cfg(cfg);
    for (int v = 0; v < (tangents ? GV_COUNT : 1); ++v)
        for (int stage = 1; stage <= 2; ++stage)
            for (int cur = 0; cur < 2; ++cur) {
                std::vector<GemmArgs<PREC>> h((size_t)np);
                for (int p = 0; p < np; ++p) {
                    // as in the single-run step: inside the two-time window the primal
                    // predictor keeps its increment and the corrector stores its field
                    const bool tan = v == GV_TANGENT, win = v == GV_PRIMAL_TAN;
                    h[(size_t)p] = make_args<PREC>(gs[(size_t)p], bs[(size_t)p], cs[(size_t)p], stage, tan, cur,
                                                   win && stage == 2, win || tan);
                    h[(size_t)p].nnt = (int)(gs[(size_t)p].C2 / tc.nt);
                    if (!x_offsets_fit<PREC>(h[(size_t)p].ldx, tc.nt, tc.kbytes)) {
                        set_error("operand pitch too large for the contraction's 32-bit offsets");
                        return TWA_EINVAL;
                    }
                }
                TWA_HIP_CHECK(hipMalloc(&pl.d_args[v][stage - 1][cur], h.size() * sizeof(GemmArgs<PREC>)));
                TWA_HIP_CHECK(hipMemcpyAsync(pl.d_args[v][stage - 1][cur], h.data(), h.size() * sizeof(GemmArgs<PREC>),
                                             hipMemcpyHostToDevice, st));
                TWA_HIP_CHECK(hipStreamSynchronize(st));   // h ends with this iteration
            }
    int dev = 0, ncu = 0;
    TWA_HIP_CHECK(hipGetDevice(&dev));
    TWA_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    int occ = 1;
    switch (cfg) {
        case 0: occ = grouped_occupancy<PREC, 0>(); break;
        case 1: occ = grouped_occupancy<PREC, 1>(); break;
        case 2: occ = grouped_occupancy<PREC, 2>(); break;
        case 3: occ = grouped_occupancy<PREC, 3>(); break;
        case 7:
            if constexpr (PREC != TWA_PREC_FP64) occ = grouped_occupancy<PREC, 7>();
            break;
        default: break;
    }
    // tile lists: (point, M tile, column tile, copy), longest contraction first
    std::vector<int> order((size_t)np);
    for (int p = 0; p < np; ++p) order[(size_t)p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return gs[(size_t)x].P > gs[(size_t)y].P; });
    for (int tl = 0; tl < (tangents ? 2 : 1); ++tl) {
        std::vector<int4> tiles;
        for (int p : order) {
            const Geometry& g = gs[(size_t)p];
            const int nnt = (int)(g.C2 / tc.nt);
            for (int mt = 0; mt < (int)g.nmt; ++mt)
                for (int nt = 0; nt < nnt; ++nt)
                    for (int cp = 0; cp < (tl ? 2 : 1); ++cp) tiles.push_back(make_int4(p, mt, nt, cp));
        }
        const int ntl = (int)tiles.size();
        const int grid = std::max(1, std::min(ncu * occ, ntl));
        xcd_permute(tiles, grid);
        TWA_HIP_CHECK(hipMalloc((void**)&pl.d_tiles[tl], tiles.size() * sizeof(int4)));
        TWA_HIP_CHECK(hipMemcpyAsync(pl.d_tiles[tl], tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice,
                                     st));
        TWA_HIP_CHECK(hipStreamSynchronize(st));   // the host list ends with this iteration
        pl.ntiles[tl] = ntl;
        pl.grid[tl] = grid;
    }
    pl.cfg = cfg;
    pl.precision = PREC;
    pl.integrator = gs[0].integrator;
    pl.tangents = tangents;
    pl.step = step;
    return TWA_OK;
}

template <int PREC>
int grouped_launch_p(const GroupedPlan& pl, int stage, int cur, int variant, hipStream_t st) {
    switch (pl.cfg) {
        case 0: return grouped_dispatch<PREC, 0>(pl, stage, cur, variant, st);
        case 1: return grouped_dispatch<PREC, 1>(pl, stage, cur, variant, st);
        case 2: return grouped_dispatch<PREC, 2>(pl, stage, cur, variant, st);
        case 3: return grouped_dispatch<PREC, 3>(pl, stage, cur, variant, st);
        case 7:
            if constexpr (PREC != TWA_PREC_FP64) return grouped_dispatch<PREC, 7>(pl, stage, cur, variant, st);
            break;
    }
    set_error("grouped launch: tile configuration must be 0..3 or 7 (not 7 in FP64)");
    return TWA_EINVAL;
}

}  // namespace twa
