// f64_core.hpp -- FP64 matrix-core tile engine for gfx950.
//
// Every dense contraction of the Cholesky J/K path (half-transforms, exchange
// products, projections, the derivative products) is a sum of products
// C[i][j] += sum_k A[i][k] B[k][j] over one output tile.  This header is the
// one tile engine they share.
//
// Matrix-core instruction: V_MFMA_F64_4X4X4_4B, four independent 4x4x4 FP64
// products per wave.  Measured on MI355X it sustains ~95% of the FP64 peak,
// far above the 16x16x4 FP64 form.  Lane mapping (measured on the device):
// for lane l, block b = (l >> 2) & 3, x = l & 3, h = l >> 4,
//     A_b[x][h] = a(l),   B_b[h][x] = b(l),   D_b[h][x] = d(l).
// The engine gives the four blocks four different 4-row groups of A and the
// SAME 4x4 piece of B, so one instruction is a 16 x 4 x 4 product:
//   A fragment (16 rows x 4 inner):  lane l holds A[row l & 15][k l >> 4]
//   B fragment (4 inner x 4 cols):   lane l holds B[k l >> 4][col l & 3]
//                                    (16 values, each read by 4 lanes)
//   output (16 x 4):                 lane l holds C[4*((l >> 2) & 3) + (l >> 4)][l & 3]
// Accumulators therefore hold distinct outputs (no cross-lane reduction) and
// a wave tile of WM x WN keeps (WM/16)*(WN/4) doubles per lane.
//
// LDS holds operand tiles in fragment order: A as [row group of 16][inner
// step of 4][64], B as [col group of 4][inner step of 4][16]; every A
// fragment read is a conflict-free 8-byte read per lane, every B fragment
// read a broadcast.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

typedef int64_t i64;

__device__ __forceinline__ double mfma4(double a, double b, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- operands
// An operand describes element (i, k) -- i the row of A or the column of B,
// k the inner index -- in two phases so that global loads stay in flight
// while the matrix cores work:
//   fetch(i, k, raw)  issues the loads of the element into raw[0..NRAW) and
//                     nothing else (addresses are clamped into range, so no
//                     branch and no wait);
//   finish(i, k, raw) combines the raw values and returns the FP64 element,
//                     0 outside the valid range.
// kContig tells the loader which index is contiguous in memory so that it
// assigns threads for coalesced reads.  Valid ranges need ni, nk >= 1.
// (Measured: a separate unchecked path for interior tiles is slower than this
// single branch-free path, because the branch splits the load schedule.)

// element (i, k) at p[i * ld + k]
struct OpKC {
    static constexpr bool kContig = true;
    static constexpr int NRAW = 1;
    const double *p;
    i64 ld;
    int ni, nk;
    __device__ __forceinline__ void fetch(int i, int k, double *raw) const
    {
        const int ic = i < ni ? i : ni - 1, kc = k < nk ? k : nk - 1;
        raw[0] = p[(i64)ic * ld + kc];
    }
    __device__ __forceinline__ double finish(int i, int k, const double *raw) const
    {
        return (i < ni && k < nk) ? raw[0] : 0.0;
    }
};

// element (i, k) at p[k * ld + i]
struct OpIC {
    static constexpr bool kContig = false;
    static constexpr int NRAW = 1;
    const double *p;
    i64 ld;
    int ni, nk;
    __device__ __forceinline__ void fetch(int i, int k, double *raw) const
    {
        const int ic = i < ni ? i : ni - 1, kc = k < nk ? k : nk - 1;
        raw[0] = p[(i64)kc * ld + ic];
    }
    __device__ __forceinline__ double finish(int i, int k, const double *raw) const
    {
        return (i < ni && k < nk) ? raw[0] : 0.0;
    }
};

// LDS layout.  A: blocks of 64 doubles per (row group of 16, inner step of 4),
// [inner 4][row 16] inside, consecutive blocks kPadA doubles apart beyond
// their 64.  B: per column group of 4, NSUB blocks of 16 doubles
// [inner 4][col 4], column groups kPadB doubles apart beyond their 16 NSUB.
// The pads break the bank conflicts of the loader's writes (four inner
// steps of one row, or sixteen column groups, written by one lane group
// would otherwise hit one bank: measured 0.5-0.9 conflicts per access); the
// fragment reads keep compile-time offsets and stay conflict-free (A) or a
// broadcast of 16 values (B).
constexpr int kPadA = 4, kPadB = 1;
constexpr int kBlkA = 64 + kPadA;

template <int NSUB>
__device__ __forceinline__ int a_slot(int r, int k)
{
    return ((r >> 4) * NSUB + (k >> 2)) * kBlkA + 16 * (k & 3) + (r & 15);
}
template <int NSUB>
__device__ __forceinline__ int b_slot(int c, int k)
{
    return (c >> 2) * (NSUB * 16 + kPadB) + (k >> 2) * 16 + 4 * (k & 3) + (c & 3);
}

// ---------------------------------------------------------------- loader
// Moves a T x BK operand tile (T rows/cols from i0, BK inner indices from k0)
// from global memory into registers (load: fetch only), then into LDS
// (store: finish, then write).  Each thread owns groups of 4 consecutive
// elements along the contiguous index.
template <int T, int BK, int NTHR, bool IS_A, class Op>
struct TileLoader {
    static constexpr int NGRP = T * BK / 4;
    static constexpr int NSTEP = (NGRP + NTHR - 1) / NTHR;
    static constexpr int NSUB = BK / 4;
    double raw[NSTEP][4][Op::NRAW];
    int i0, k0;

    __device__ __forceinline__ void coords(int g, int e, int &i, int &k) const
    {
        if (Op::kContig) {
            i = i0 + g / (BK / 4);
            k = k0 + (g % (BK / 4)) * 4 + e;
        } else {
            k = k0 + g / (T / 4);
            i = i0 + (g % (T / 4)) * 4 + e;
        }
    }

    __device__ __forceinline__ void load(const Op &op, int i0_, int k0_, int tid)
    {
        i0 = i0_;
        k0 = k0_;
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            int g = tid + s * NTHR;
            if (NGRP % NTHR == 0 || g < NGRP) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int i, k;
                    coords(g, e, i, k);
                    op.fetch(i, k, raw[s][e]);
                }
            }
        }
    }

    __device__ __forceinline__ void store(const Op &op, double *lds, int tid) const
    {
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            int g = tid + s * NTHR;
            if (NGRP % NTHR == 0 || g < NGRP) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int i, k;
                    coords(g, e, i, k);
                    const double v = op.finish(i, k, raw[s][e]);
                    const int li = i - i0, lk = k - k0;
                    lds[IS_A ? a_slot<NSUB>(li, lk) : b_slot<NSUB>(li, lk)] = v;
                }
            }
        }
    }
};

// ---------------------------------------------------------------- tile GEMM
// One workgroup computes a BM x BN output tile with inner stages of BK;
// waves are laid out (BM/WM) x (BN/WN), each owning a WM x WN sub-tile.
template <int BM_, int BN_, int WM, int WN, int BK>
struct Tile {
    static constexpr bool kMfma16 = false;
    static constexpr int BM = BM_, BN = BN_;
    static constexpr int WROWS = BM / WM, WCOLS = BN / WN;
    static constexpr int NWAVE = WROWS * WCOLS;
    static constexpr int NTHR = NWAVE * 64;
    static constexpr int MA = WM / 16, NB = WN / 4, NSUB = BK / 4;
    static constexpr int BGRP = NSUB * 16 + kPadB;              // doubles per B column group
    static constexpr int A_DOUBLES = (BM / 16) * NSUB * kBlkA, B_DOUBLES = (BN / 4) * BGRP;
    static constexpr int LDS_DOUBLES = 2 * (A_DOUBLES + B_DOUBLES);
    static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 4 == 0, "tile");
    static_assert(BK % 4 == 0 && BM % 16 == 0 && BN % 4 == 0, "tile");
};

template <class TL>
struct Acc {
    double c[TL::MA][TL::NB];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < TL::MA; i++)
#pragma unroll
            for (int j = 0; j < TL::NB; j++)
                c[i][j] = 0.0;
    }
};

// acc += sum over k in [k_begin, k_end) of A(m0 + i, k) * B(n0 + j, k).
// lds must hold TL::LDS_DOUBLES doubles.  Every thread of the workgroup calls
// this.  Operands return 0 outside their valid range.
//
// Pipeline: two LDS stage buffers; the global loads of stage kt + 1 are
// issued before the matrix-core work of stage kt and written to the other
// buffer after it, one barrier per stage.
template <class TL, class OA, class OB>
__device__ __forceinline__ void tile_gemm(const OA &A, const OB &B, int m0, int n0, int k_begin,
                                          int k_end, double *lds, Acc<TL> &acc)
{
    constexpr int BK = TL::NSUB * 4;
    constexpr int BM = TL::WROWS * TL::MA * 16, BN = TL::WCOLS * TL::NB * 4;
    // Stage buffer s starts at lds + s * STAGE: A tile, then B tile.  Plain
    // pointer arithmetic keeps every access an LDS (ds_*) instruction.
    constexpr int STAGE = TL::A_DOUBLES + TL::B_DOUBLES;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int boff = 4 * (lane >> 4) + (lane & 3);

    TileLoader<BM, BK, TL::NTHR, true, OA> la;
    TileLoader<BN, BK, TL::NTHR, false, OB> lb;
    const int nk = (k_end - k_begin + BK - 1) / BK;
    if (nk <= 0)
        return;
    la.load(A, m0, k_begin, tid);
    lb.load(B, n0, k_begin, tid);
    la.store(A, lds, tid);
    lb.store(B, lds + TL::A_DOUBLES, tid);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
        const int cur = kt & 1;
        const bool more = (kt + 1) < nk;
        if (more) {
            la.load(A, m0, k_begin + (kt + 1) * BK, tid);
            lb.load(B, n0, k_begin + (kt + 1) * BK, tid);
        }
        const double *pa = lds + cur * STAGE + (wr * TL::MA) * TL::NSUB * kBlkA + lane;
        const double *pb = lds + cur * STAGE + TL::A_DOUBLES + (wc * TL::NB) * TL::BGRP + boff;
#pragma unroll
        for (int s = 0; s < TL::NSUB; s++) {
            double a[TL::MA], b[TL::NB];
#pragma unroll
            for (int i = 0; i < TL::MA; i++)
                a[i] = pa[(i * TL::NSUB + s) * kBlkA];
#pragma unroll
            for (int j = 0; j < TL::NB; j++)
                b[j] = pb[j * TL::BGRP + s * 16];
#pragma unroll
            for (int i = 0; i < TL::MA; i++)
#pragma unroll
                for (int j = 0; j < TL::NB; j++)
                    acc.c[i][j] = mfma4(a[i], b[j], acc.c[i][j]);
        }
        if (more) {
            la.store(A, lds + (cur ^ 1) * STAGE, tid);
            lb.store(B, lds + (cur ^ 1) * STAGE + TL::A_DOUBLES, tid);
        }
        __syncthreads();
    }
}

// acc += sum over segments s < nseg of sum over k in [0, kdepth) of
// A_s(m0 + i, k) * B_s(n0 + j, k), where operand A_s is A with its base moved
// by s * segA elements (B_s likewise).  The stages of all segments form one
// pipeline: the first stage of segment s + 1 is loaded while the last stage
// of segment s is multiplied, so a workgroup that sums products over many
// slabs never drains between them.  Operands must not use p in finish().
template <class TL, class OA, class OB>
__device__ __forceinline__ void tile_gemm_seg(const OA &A, const OB &B, i64 segA, i64 segB,
                                              int nseg, int m0, int n0, int kdepth, double *lds,
                                              Acc<TL> &acc)
{
    constexpr int BK = TL::NSUB * 4;
    constexpr int BM = TL::WROWS * TL::MA * 16, BN = TL::WCOLS * TL::NB * 4;
    constexpr int STAGE = TL::A_DOUBLES + TL::B_DOUBLES;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int boff = 4 * (lane >> 4) + (lane & 3);

    TileLoader<BM, BK, TL::NTHR, true, OA> la;
    TileLoader<BN, BK, TL::NTHR, false, OB> lb;
    const int nk = (kdepth + BK - 1) / BK;
    const int total = nk * nseg;
    if (total <= 0)
        return;
    auto opA = [&](int g) {
        OA a = A;
        a.p += (i64)(g / nk) * segA;
        return a;
    };
    auto opB = [&](int g) {
        OB b = B;
        b.p += (i64)(g / nk) * segB;
        return b;
    };
    la.load(opA(0), m0, 0, tid);
    lb.load(opB(0), n0, 0, tid);
    la.store(A, lds, tid);
    lb.store(B, lds + TL::A_DOUBLES, tid);
    __syncthreads();
    for (int g = 0; g < total; g++) {
        const int cur = g & 1;
        const bool more = (g + 1) < total;
        if (more) {
            const int kn = ((g + 1) % nk) * BK;
            la.load(opA(g + 1), m0, kn, tid);
            lb.load(opB(g + 1), n0, kn, tid);
        }
        const double *pa = lds + cur * STAGE + (wr * TL::MA) * TL::NSUB * kBlkA + lane;
        const double *pb = lds + cur * STAGE + TL::A_DOUBLES + (wc * TL::NB) * TL::BGRP + boff;
#pragma unroll
        for (int s = 0; s < TL::NSUB; s++) {
            double a[TL::MA], b[TL::NB];
#pragma unroll
            for (int i = 0; i < TL::MA; i++)
                a[i] = pa[(i * TL::NSUB + s) * kBlkA];
#pragma unroll
            for (int j = 0; j < TL::NB; j++)
                b[j] = pb[j * TL::BGRP + s * 16];
#pragma unroll
            for (int i = 0; i < TL::MA; i++)
#pragma unroll
                for (int j = 0; j < TL::NB; j++)
                    acc.c[i][j] = mfma4(a[i], b[j], acc.c[i][j]);
        }
        if (more) {
            la.store(A, lds + (cur ^ 1) * STAGE, tid);
            lb.store(B, lds + (cur ^ 1) * STAGE + TL::A_DOUBLES, tid);
        }
        __syncthreads();
    }
}

// Calls f(row, col, value) for every output element this lane holds:
// accumulator (i, j) is element (m0 + wr*WM + 16i + 4*((lane >> 2) & 3) +
// (lane >> 4), n0 + wc*WN + 4j + (lane & 3)).
template <class TL, class F>
__device__ __forceinline__ void tile_foreach(const Acc<TL> &acc, int m0, int n0, F &&f)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int rb = m0 + wr * (TL::MA * 16) + 4 * ((lane >> 2) & 3) + (lane >> 4);
    const int cb = n0 + wc * (TL::NB * 4) + (lane & 3);
#pragma unroll
    for (int i = 0; i < TL::MA; i++)
#pragma unroll
        for (int j = 0; j < TL::NB; j++)
            f(rb + 16 * i, cb + 4 * j, acc.c[i][j]);
}

// Workgroup index remapped so that consecutive logical tiles land on the same
// XCD (the hardware deals workgroups round-robin over the 8 XCDs, each with
// its own L2): over the first 8 (n / 8) indices, logical = xcd * (n / 8) +
// hw / 8; the last n % 8 keep their index.
__device__ __forceinline__ int xcd_swizzle(int hw, int n)
{
    const int q = n >> 3;
    if (hw >= 8 * q)
        return hw;
    return (hw & 7) * q + (hw >> 3);
}

} // namespace jk
