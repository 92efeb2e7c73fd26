// f64_core.hpp -- FP64 matrix-core tile engine for gfx950.
//
// Every dense contraction of the Cholesky J/K path (half-transforms, exchange
// products, projections, the derivative products) is a sum of products
// C[i][j] += sum_k A[i][k] B[k][j] over one tile.  This header provides the
// one tile engine they share.
//
// Matrix-core instruction: V_MFMA_F64_4X4X4_4B (four independent 4x4x4 FP64
// products per wave).  Measured on MI355X it sustains ~95% of the FP64 peak,
// well above the 16x16x4 FP64 form.  Lane mapping, measured on the device:
// for lane l, block b = (l >> 2) & 3, x = l & 3, h = l >> 4,
//     A_b[x][h] = a(l),   B_b[h][x] = b(l),   D_b[h][x] = d(l).
// The engine uses the four blocks as a split of a 16-long inner step:
// block b covers inner indices 4b .. 4b+3, so one instruction adds a 4x4
// output tile over 16 inner indices, kept as four partial tiles (one per
// block) that are summed once, at the end, by two lane exchanges.
//
// Fragment of an operand tile of 4 rows (A) or 4 columns (B) by 16 inner
// indices: lane l holds element (x = l & 3, k = 4*((l >> 2) & 3) + (l >> 4)).
// Inverse: element (x, k) sits in lane 16*(k & 3) + 4*(k >> 2) + x.
// LDS holds operand tiles in this fragment order, 64 doubles per fragment, so
// every fragment read is one conflict-free 8-byte LDS read per lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

typedef int64_t i64;

__device__ __forceinline__ double mfma4(double a, double b, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int frag_slot(int x, int k)
{
    return 16 * (k & 3) + 4 * (k >> 2) + x;
}

// ---------------------------------------------------------------- operands
// An operand accessor returns element (i, k) -- i the row of A or the column
// of B, k the inner index -- as an FP64 value, 0 outside the valid range.
// kContig tells the loader which index is contiguous in memory so that it
// assigns threads for coalesced reads.

// element (i, k) at p[i * ld + k]
struct OpKC {
    static constexpr bool kContig = true;
    const double *p;
    i64 ld;
    int ni, nk;
    __device__ double operator()(int i, int k) const
    {
        return (i < ni && k < nk) ? p[(i64)i * ld + k] : 0.0;
    }
};

// element (i, k) at p[k * ld + i]
struct OpIC {
    static constexpr bool kContig = false;
    const double *p;
    i64 ld;
    int ni, nk;
    __device__ double operator()(int i, int k) const
    {
        return (i < ni && k < nk) ? p[(i64)k * ld + i] : 0.0;
    }
};

// ---------------------------------------------------------------- loader
// Moves a T x 16 operand tile (T rows/cols, 16 inner indices starting at k0,
// i starting at i0) from global memory into registers, then into LDS in
// fragment order.  Each thread owns groups of 4 consecutive elements along
// the contiguous index.
template <int T, int NTHR, class Op>
struct TileLoader {
    static constexpr int NGRP = 4 * T;                       // groups of 4
    static constexpr int NSTEP = (NGRP + NTHR - 1) / NTHR;
    double v[NSTEP][4];

    __device__ __forceinline__ void load(const Op &op, int i0, int k0, int tid)
    {
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            int g = tid + s * NTHR;
            if (NGRP % NTHR == 0 || g < NGRP) {
                if (Op::kContig) {
                    int i = g >> 2, kq = (g & 3) * 4;
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        v[s][e] = op(i0 + i, k0 + kq + e);
                } else {
                    int k = g / (T / 4), iq = (g % (T / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        v[s][e] = op(i0 + iq + e, k0 + k);
                }
            }
        }
    }

    __device__ __forceinline__ void store(double *lds, int tid) const
    {
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            int g = tid + s * NTHR;
            if (NGRP % NTHR == 0 || g < NGRP) {
                if (Op::kContig) {
                    int i = g >> 2, kq = (g & 3) * 4;
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        lds[(i >> 2) * 64 + frag_slot(i & 3, kq + e)] = v[s][e];
                } else {
                    int k = g / (T / 4), iq = (g % (T / 4)) * 4;
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        lds[(iq >> 2) * 64 + frag_slot(e, k)] = v[s][e];
                }
            }
        }
    }
};

// ---------------------------------------------------------------- tile GEMM
// One workgroup computes a BM x BN output tile; waves are laid out
// (BM/WM) x (BN/WN), each wave owning a WM x WN sub-tile held as
// (WM/4) x (WN/4) accumulators (one double per lane each, four partial tiles
// per accumulator).  LDS: 2 * (BM + BN) * 16 doubles.
template <int BM, int BN, int WM, int WN>
struct Tile {
    static constexpr int WROWS = BM / WM, WCOLS = BN / WN;
    static constexpr int NWAVE = WROWS * WCOLS;
    static constexpr int NTHR = NWAVE * 64;
    static constexpr int MA = WM / 4, NB = WN / 4;
    static constexpr int LDS_DOUBLES = 2 * (BM + BN) * 16;
    static_assert(BM % WM == 0 && BN % WN == 0 && WM % 4 == 0 && WN % 4 == 0, "tile");
};

template <int BM, int BN, int WM, int WN>
struct Acc {
    double c[WM / 4][WN / 4];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < WM / 4; i++)
#pragma unroll
            for (int j = 0; j < WN / 4; j++)
                c[i][j] = 0.0;
    }
    // Sum the four per-block partial tiles; afterwards every lane of a block
    // group holds the full value of its element.
    __device__ __forceinline__ void reduce_blocks()
    {
#pragma unroll
        for (int i = 0; i < WM / 4; i++)
#pragma unroll
            for (int j = 0; j < WN / 4; j++) {
                double t = c[i][j];
                t += __shfl_xor(t, 4);
                t += __shfl_xor(t, 8);
                c[i][j] = t;
            }
    }
};

// Accumulate sum over k in [0, kdim) of A(m0 + i, k) * B(n0 + j, k) into acc.
// lds must hold Tile::LDS_DOUBLES doubles.  All threads of the workgroup
// must call this.
template <int BM, int BN, int WM, int WN, class OA, class OB>
__device__ __forceinline__ void tile_gemm(const OA &A, const OB &B, int m0, int n0, int kdim,
                                          double *lds, Acc<BM, BN, WM, WN> &acc)
{
    typedef Tile<BM, BN, WM, WN> TL;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    double *ldsA[2] = {lds, lds + (BM + BN) * 16};
    double *ldsB[2] = {lds + BM * 16, lds + (BM + BN) * 16 + BM * 16};

    TileLoader<BM, TL::NTHR, OA> la;
    TileLoader<BN, TL::NTHR, OB> lb;
    const int nk = (kdim + 15) / 16;
    if (nk == 0)
        return;
    la.load(A, m0, 0, tid);
    lb.load(B, n0, 0, tid);
    la.store(ldsA[0], tid);
    lb.store(ldsB[0], tid);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
        const int cur = kt & 1;
        const bool more = (kt + 1) < nk;
        if (more) {
            la.load(A, m0, (kt + 1) * 16, tid);
            lb.load(B, n0, (kt + 1) * 16, tid);
        }
        double a[TL::MA], b[TL::NB];
        const double *pa = ldsA[cur] + (wr * TL::MA) * 64 + lane;
        const double *pb = ldsB[cur] + (wc * TL::NB) * 64 + lane;
#pragma unroll
        for (int i = 0; i < TL::MA; i++)
            a[i] = pa[i * 64];
#pragma unroll
        for (int j = 0; j < TL::NB; j++)
            b[j] = pb[j * 64];
#pragma unroll
        for (int i = 0; i < TL::MA; i++)
#pragma unroll
            for (int j = 0; j < TL::NB; j++)
                acc.c[i][j] = mfma4(a[i], b[j], acc.c[i][j]);
        if (more) {
            la.store(ldsA[cur ^ 1], tid);
            lb.store(ldsB[cur ^ 1], tid);
        }
        __syncthreads();
    }
}

// After acc.reduce_blocks(): the element held by this lane for accumulator
// (i, j) is output (row, col) = (m0 + wr*WM + 4i + (lane >> 4),
// n0 + wc*WN + 4j + (lane & 3)).  Lanes of block b = (lane >> 2) & 3 write
// the accumulators with (j & 3) == b, so every lane writes and each element
// is written once.
template <int BM, int BN, int WM, int WN, class F>
__device__ __forceinline__ void tile_foreach(const Acc<BM, BN, WM, WN> &acc, int m0, int n0, F &&f)
{
    typedef Tile<BM, BN, WM, WN> TL;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int blk = (lane >> 2) & 3;
    const int rb = m0 + wr * WM + (lane >> 4);
    const int cb = n0 + wc * WN + (lane & 3);
#pragma unroll
    for (int i = 0; i < TL::MA; i++)
#pragma unroll
        for (int j = 0; j < TL::NB; j++)
            if ((j & 3) == blk)
                f(rb + 4 * i, cb + 4 * j, acc.c[i][j]);
}

// Workgroup index remapped so that consecutive logical tiles land on the same
// XCD (the hardware deals workgroups round-robin over the 8 XCDs, each with
// its own L2): logical = xcd * ceil(n/8) + (hw / 8), folded back into range.
__device__ __forceinline__ int xcd_swizzle(int hw, int n)
{
    const int per = (n + 7) / 8;
    const int xcd = hw & 7, slot = hw >> 3;
    int logical = xcd * per + slot;
    // Grids that are not a multiple of 8 leave holes; fall back to identity
    // for them to keep the map a bijection.
    return (n % 8 == 0) ? logical : hw;
}

} // namespace jk
