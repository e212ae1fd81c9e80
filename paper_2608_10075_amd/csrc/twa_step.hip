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
#include "twa_internal.h"
#include "twa_device.h"

namespace twa {

template <int PREC>
struct GemmArgs {
    typedef typename Prec<PREC>::G G;
    typedef typename Prec<PREC>::S S;
    const G* A;
    int64_t lda;        // elements
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
    G* Xnext;           // stage 2 writes (s-part, ld 2P for primal, P for tangents)
    int64_t ldxn;
    const S* part_prim; // primal partial sums read by the epilogue
    S* part_out;        // partial sums written
    const S* g;
    int store_y2;
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
};

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

// ---------------------------------------------------------------------------
// contraction + fused Heun stage
template <int PREC, int MT, int NT, int KB, int WMW, int WNW, int NST, int STAGE, bool TAN>
__global__ __launch_bounds__(64 * WMW * WNW) void heun_stage_kernel(GemmArgs<PREC> a) {
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
    __shared__ S red[WMW][NTRJ][3];

    // XCD-aware tile order: workgroups are dispatched round-robin over the 8
    // XCDs, so workgroup b runs on XCD b % 8.  Each XCD is given a contiguous
    // range of tiles ordered M-tile-major, so the workgroups resident on one
    // XCD share the same rows of A (and walk K together) in that XCD's L2.
    int mt, nt;
    {
        const int nnt = a.nnt;            // column tiles
        const int T = (int)gridDim.x;     // total tiles = nmt * nnt
        const int q = T / 8, r = T % 8;
        const int b = (int)blockIdx.x, x = b % 8, j = b / 8;
        const int L = x * q + (x < r ? x : r) + j;
        mt = L / nnt;
        nt = L % nnt;
    }
    const int cp = blockIdx.z;
    const int64_t m0 = (int64_t)mt * MT, n0 = (int64_t)nt * NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WMW, wn = wave / WMW;
    const int wm0 = wm * WM, wn0 = wn * WN;
    const int64_t P = a.P, Bp = a.Bp, nmt = a.nmt;
    const int64_t k0t = n0 / 2;    // first trajectory of the tile

    // ---- collective sums of this tile's trajectories (ordered over M tiles)
    for (int t = tid; t < NTRJ; t += NTHR) {
        const int64_t k = k0t + t;
        const S* pp = a.part_prim;
        S sx = 0, sy = 0;
        for (int64_t q = 0; q < nmt; ++q) {
            sx += pp[(0 * nmt + q) * Bp + k];
            sy += pp[(1 * nmt + q) * Bp + k];
        }
        sS[t][0] = sx;
        sS[t][1] = sy;
        sG[t][0] = a.g[k];
        sG[t][1] = a.g[Bp + k];
        if constexpr (TAN) {
            const S* tp = a.tpart_in + cp * a.t_part_copy;
            S tx = 0, ty = 0;
            for (int64_t q = 0; q < nmt; ++q) {
                tx += tp[(0 * nmt + q) * Bp + k];
                ty += tp[(1 * nmt + q) * Bp + k];
            }
            sT[t][0] = tx;
            sT[t][1] = ty;
        }
    }

    // ---- main loop: acc[i][col] = sum_k A[m0+i][k] X[n0+col][k]
    AV acc[BI][BJ];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) acc[i][j] = AV{0, 0, 0, 0};

    const char* Ag = reinterpret_cast<const char*>(a.A + m0 * a.lda);
    const char* Xg = reinterpret_cast<const char*>(a.X + cp * a.x_copy + n0 * a.ldx);
    const int64_t lda_b = a.lda * (int64_t)sizeof(G), ldx_b = a.ldx * (int64_t)sizeof(G);
    const int nk = (int)(a.K / KT);
    // Direct global -> LDS loads (global_load_lds_dwordx4): one wave
    // instruction moves 64 x 16 bytes into 1 KB of LDS, lane i to offset 16 i,
    // so each lane fetches the global piece that belongs at its slot.
    constexpr int RPC = 1024 / KB;                 // rows per 1 KB chunk
    constexpr int NCH = (MT + NT) / RPC;           // chunks per stage
    constexpr int NWV = NTHR / 64;
    constexpr int CPW = NCH / NWV;                 // chunks per wave per stage
    static_assert(NCH % NWV == 0 && MT % RPC == 0, "chunking");
    auto swz = [](int r16) { return (r16 / (16 / PCS)) % PCS; };
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const char* src[CPW];
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
        const int q = wv + j * NWV;
        const int row = q * RPC + lane / PCS;
        const int pc = (lane % PCS) ^ swz(row & 15);
        src[j] = row < MT ? Ag + row * lda_b + pc * 16 : Xg + (int64_t)(row - MT) * ldx_b + pc * 16;
    }
    typedef __attribute__((address_space(3))) char lds_t;
    typedef const __attribute__((address_space(1))) void gptr_t;
#define TWA_DMA(KT_, BUF_)                                                                              \
    do {                                                                                                \
        const int64_t kofs_ = (int64_t)(KT_) * KB;                                                      \
        _Pragma("unroll") for (int j = 0; j < CPW; ++j) __builtin_amdgcn_global_load_lds(               \
            (gptr_t*)(src[j] + kofs_), (lds_t*)((BUF_) + (wv + j * NWV) * 1024), 16, 0, 0);              \
    } while (0)

    // fragment read offsets of this lane (row within a 16-row block, swizzle)
    const int ra = Prec<PREC>::arow(lane & 15), rx = lane & 15;
    const int offA = (wm0 + ra) * KB, offX = (MT + wn0 + rx) * KB;
    const int swA = swz(ra), swX = swz(rx), grp = lane >> 4;
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
                if (nk - 1 - kt >= NST - 2) TWA_WAIT_VM((NST - 2) * CPW);
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
#pragma unroll
    for (int p = 0; p < BJ / 2; ++p) {
        const int kl = wn0 / 2 + 16 * p + (lane & 15);
        const int64_t k = k0t + kl;
        const S Sx = sS[kl][0], Sy = sS[kl][1];
        const S hx0 = c1 * Sx + c2 * sG[kl][0];
        const S hy0 = c1 * Sy + c2 * sG[kl][1];
        S ps0 = 0, ps1 = 0, ps2 = 0;
#pragma unroll
        for (int bi = 0; bi < BI; ++bi) {
            const int64_t i0 = m0 + wm0 + 16 * bi + 4 * (lane >> 4);
            const int64_t off = k * P + i0;
            S x[4], y[4], z[4];
            ld4(a.s_cur + off, x);
            ld4(a.s_cur + SP + off, y);
            ld4(a.s_cur + 2 * SP + off, z);
            if constexpr (!TAN && STAGE == 1) {
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
                st4(a.dlt + off, dx);
                st4(a.dlt + SP + off, dy);
                st4(a.dlt + 2 * SP + off, dz);
                st4(a.Y + off, yx);
                st4(a.Y + SP + off, yy);
                stg4<PREC>(a.Dop + opcol(k, 0) * P + i0, dx);
                stg4<PREC>(a.Dop + opcol(k, 1) * P + i0, dy);
            } else if constexpr (!TAN && STAGE == 2) {
                S dx[4], dy[4], dz[4], yx[4], yy[4], nx[4], ny[4], nz[4];
                ld4(a.dlt + off, dx);
                ld4(a.dlt + SP + off, dy);
                ld4(a.dlt + 2 * SP + off, dz);
                ld4(a.Y + off, yx);
                ld4(a.Y + SP + off, yy);
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
                st4(a.s_next + off, nx);
                st4(a.s_next + SP + off, ny);
                st4(a.s_next + 2 * SP + off, nz);
                if (a.store_y2) {
                    st4(a.Y + off, yx);
                    st4(a.Y + SP + off, yy);
                }
                stg4<PREC>(a.Xnext + opcol(k, 0) * a.ldxn + i0, nx);
                stg4<PREC>(a.Xnext + opcol(k, 1) * a.ldxn + i0, ny);
            } else if constexpr (TAN && STAGE == 1) {
                const S tSx = sT[kl][0], tSy = sT[kl][1];
                const S* tc = a.t_cur + cp * a.t_state_copy;
                S u[4], v[4], w[4], yx[4], yy[4], ex[4], ey[4], ez[4], ax4[4], ay4[4];
                ld4(tc + off, u);
                ld4(tc + SP + off, v);
                ld4(tc + 2 * SP + off, w);
                ld4(a.Y + off, yx);
                ld4(a.Y + SP + off, yy);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S Hx = yx[r] + hx0, Hy = yy[r] + hy0;
                    const S ax = acc[bi][2 * p][r], ay = acc[bi][2 * p + 1][r];
                    const S dHx = ax + c1 * tSx, dHy = ay + c1 * tSy;
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
                stg4<PREC>(tdo + opcol(k, 0) * P + i0, ex);
                stg4<PREC>(tdo + opcol(k, 1) * P + i0, ey);
            } else {  // TAN && STAGE == 2
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
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const S px = x[r] + dx[r], py = y[r] + dy[r], pz = z[r] + dz[r];
                    const S Hx = yx[r] + hx0, Hy = yy[r] + hy0;
                    const S pu = u[r] + du[r], pv = v[r] + dv[r], pw = w[r] + dw[r];
                    const S dHx = tyx[r] + acc[bi][2 * p][r] + c1 * tSx;
                    const S dHy = tyy[r] + acc[bi][2 * p + 1][r] + c1 * tSy;
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
                stg4<PREC>(txo + opcol(k, 0) * a.ldxn + i0, nu);
                stg4<PREC>(txo + opcol(k, 1) * a.ldxn + i0, nv);
            }
        }
        // partial spin sums of the new values: lanes sharing a trajectory,
        // then waves along M, in a fixed order
        ps0 += __shfl_xor(ps0, 16);
        ps1 += __shfl_xor(ps1, 16);
        ps2 += __shfl_xor(ps2, 16);
        ps0 += __shfl_xor(ps0, 32);
        ps1 += __shfl_xor(ps1, 32);
        ps2 += __shfl_xor(ps2, 32);
        if (lane < 16) {
            red[wm][kl][0] = ps0;
            red[wm][kl][1] = ps1;
            red[wm][kl][2] = ps2;
        }
    }
    __syncthreads();
    S* po = a.part_out + (TAN ? cp * a.t_part_copy : 0);
    for (int t = tid; t < 3 * NTRJ; t += NTHR) {
        const int c = t / NTRJ, kl = t % NTRJ;
        S s = 0;
#pragma unroll
        for (int q = 0; q < WMW; ++q) s += red[q][kl][c];
        po[((int64_t)c * nmt + mt) * Bp + k0t + kl] = s;
    }
    if constexpr (!TAN && STAGE == 2) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && tid == 0) a.step[0] += 1;
    }
}

// ---------------------------------------------------------------------------
// tile configurations
static const TileCfg kCfgs[] = {
    {0, 16, 32, 64, 1, 1, 2, "16x32 K64B 1w 2st"},
    {1, 64, 64, 64, 2, 2, 4, "64x64 K64B 4w 4st"},
    {2, 128, 128, 128, 2, 2, 4, "128x128 K128B 4w 4st"},
    {3, 128, 128, 64, 2, 2, 8, "128x128 K64B 4w 8st"},
    {4, 256, 128, 64, 4, 1, 6, "256x128 K64B 4w 6st"},
    {5, 128, 256, 64, 2, 2, 6, "128x256 K64B 4w 6st"},
    {6, 256, 256, 64, 4, 2, 4, "256x256 K64B 8w 4st"},
};
int n_tile_cfgs() { return (int)(sizeof(kCfgs) / sizeof(kCfgs[0])); }
const TileCfg& tile_cfg(int id) { return kCfgs[id]; }

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
TWA_CFG(6, 256, 256, 64, 4, 2, 4)

template <int PREC, int CFG>
static int launch_gemm_t(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage,
                         bool tangent, int cur, bool store_y2, hipStream_t st) {
    typedef CfgT<PREC, CFG> C;
    typedef typename Prec<PREC>::G G;
    typedef typename Prec<PREC>::S S;
    GemmArgs<PREC> a{};
    const int64_t P = g.P, Bp = g.Bp;
    a.A = static_cast<const G*>(b.A);
    a.lda = 2 * P;
    a.P = P;
    a.Bp = Bp;
    a.nmt = g.nmt;
    a.c1 = (S)c.c1;
    a.c2 = (S)c.c2;
    a.s_cur = static_cast<const S*>(b.s[cur]);
    a.s_next = static_cast<S*>(b.s[1 - cur]);
    a.dlt = static_cast<S*>(b.dlt);
    a.Y = static_cast<S*>(b.Y);
    a.Dop = static_cast<G*>(b.Dop);
    a.g = static_cast<const S*>(b.g);
    a.store_y2 = store_y2 ? 1 : 0;
    a.step = b.step;
    const int64_t SP3 = 3 * Bp * P;
    a.t_state_copy = SP3;
    a.t_y_copy = 2 * Bp * P;
    a.t_part_copy = 3 * g.nmt * Bp;
    a.t_op_copy = g.C2 * P;
    int ncopy = 1;
    if (!tangent) {
        if (stage == 1) {
            a.X = static_cast<const G*>(b.Xop);
            a.ldx = 2 * P;
            a.K = 2 * P;
            a.part_prim = static_cast<const S*>(b.part[0]);
            a.part_out = static_cast<S*>(b.part[1]);
        } else {
            a.X = static_cast<const G*>(b.Dop);
            a.ldx = P;
            a.K = P;
            a.part_prim = static_cast<const S*>(b.part[1]);
            a.part_out = static_cast<S*>(b.part[0]);
            a.Xnext = static_cast<G*>(b.Xop);
            a.ldxn = 2 * P;
        }
    } else {
        ncopy = 2;
        a.t_cur = static_cast<const S*>(b.ts[cur]);
        a.t_next = static_cast<S*>(b.ts[1 - cur]);
        a.t_dlt = static_cast<S*>(b.tdlt);
        a.tY = static_cast<S*>(b.tY);
        a.tDop = static_cast<G*>(b.tDop);
        a.x_copy = g.C2 * P;
        a.K = P;
        a.ldx = P;
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
            a.ldxn = P;
        }
    }
    // grid.x enumerates all (M tile, column tile) pairs; each block derives its tile
    a.nnt = (int)(g.C2 / C::NT);
    dim3 grid((unsigned)((P / C::MT) * (g.C2 / C::NT)), 1u, (unsigned)ncopy);
    dim3 block(64 * C::WMW * C::WNW);
    if (stage == 1) {
        if (tangent)
            hipLaunchKernelGGL((heun_stage_kernel<PREC, C::MT, C::NT, C::KB, C::WMW, C::WNW, C::NST, 1, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((heun_stage_kernel<PREC, C::MT, C::NT, C::KB, C::WMW, C::WNW, C::NST, 1, false>), grid, block, 0, st, a);
    } else {
        if (tangent)
            hipLaunchKernelGGL((heun_stage_kernel<PREC, C::MT, C::NT, C::KB, C::WMW, C::WNW, C::NST, 2, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((heun_stage_kernel<PREC, C::MT, C::NT, C::KB, C::WMW, C::WNW, C::NST, 2, false>), grid, block, 0, st, a);
    }
    TWA_HIP_CHECK(hipGetLastError());
    return TWA_OK;
}

template <int PREC>
static int launch_gemm_p(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage,
                         bool tangent, int cur, bool store_y2, hipStream_t st) {
    switch (g.cfg) {
        case 0: return launch_gemm_t<PREC, 0>(g, b, c, stage, tangent, cur, store_y2, st);
        case 1: return launch_gemm_t<PREC, 1>(g, b, c, stage, tangent, cur, store_y2, st);
        case 2: return launch_gemm_t<PREC, 2>(g, b, c, stage, tangent, cur, store_y2, st);
        case 3: return launch_gemm_t<PREC, 3>(g, b, c, stage, tangent, cur, store_y2, st);
    }
    if constexpr (PREC != TWA_PREC_FP64) {
        switch (g.cfg) {
            case 4: return launch_gemm_t<PREC, 4>(g, b, c, stage, tangent, cur, store_y2, st);
            case 5: return launch_gemm_t<PREC, 5>(g, b, c, stage, tangent, cur, store_y2, st);
            case 6: return launch_gemm_t<PREC, 6>(g, b, c, stage, tangent, cur, store_y2, st);
        }
    }
    set_error("unknown tile configuration");
    return TWA_EINVAL;
}

int launch_gemm(const Geometry& g, const EnsembleBuffers& b, const StepConsts& c, int stage, bool tangent,
                int cur, bool store_y2, hipStream_t st) {
    switch (g.precision) {
        case TWA_PREC_FP64: return launch_gemm_p<TWA_PREC_FP64>(g, b, c, stage, tangent, cur, store_y2, st);
        case TWA_PREC_FP32: return launch_gemm_p<TWA_PREC_FP32>(g, b, c, stage, tangent, cur, store_y2, st);
        case TWA_PREC_BF16: return launch_gemm_p<TWA_PREC_BF16>(g, b, c, stage, tangent, cur, store_y2, st);
        case TWA_PREC_FP16: return launch_gemm_p<TWA_PREC_FP16>(g, b, c, stage, tangent, cur, store_y2, st);
    }
    set_error("unknown precision");
    return TWA_EINVAL;
}

}  // namespace twa
