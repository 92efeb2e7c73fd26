// slice_core.hpp -- fixed-point slice products on gfx950 INT8 matrix cores.
//
// Split-precision scheme of the mixed J/K path.  Every FP64 row a[0..n) of an
// operand gets one power-of-two scale 2^e with max|a| <= 2^e * 127/128, and
// each element is rounded to the 31-bit integer N = rint(a 2^(31 - e)),
// |N| <= 127 * 2^24, written as NS = 4 balanced base-256 digits
//     N = d1 2^24 + d2 2^16 + d3 2^8 + d4,   d2..d4 in [-128, 127],
// taken from the bottom (d4 = ((N + 128) mod 256) - 128, then N -> (N - d4)/256,
// ...); the leading digit is what remains, |d1| <= 127.  So
//     a = 2^(e - 7) * sum_{i=1..4} d_i 2^(-8 (i - 1)) + rest,  |rest| <= 2^(e - 32).
// A product of two rows is
//     sum_k a_k b_k = 2^(ea + eb - 14) * sum_{l=2..L} 2^(-8 (l - 2)) * S_l,
//     S_l = sum_{i+j=l} sum_k d_i(a_k) d_j(b_k),
// keeping the 13 digit pairs with i + j <= L = 6.  Each S_l is an exact
// integer: the matrix cores multiply int8 digits and accumulate in int32; a
// level holds at most 4 pairs of |d_i d_j| <= 2^14 per inner index, so
// |S_l| <= 2^16 n < 2^31 for n <= kSliceMaxDepth = 32767 inner indices per
// accumulation (enforced by the planner).  The levels are combined in FP64
// with power-of-two weights, so the only approximations are the rounding of
// N (relative 2^-32 of the row scale), the three dropped pairs, and FP64
// rounding of the combination.
//
// Instruction: V_MFMA_I32_32X32X32_I8.  Lane layout (measured on the device):
// lane l holds A[row l % 32][k 16*(l/32) .. +15] and B[k 16*(l/32) .. +15][col
// l % 32] as 16 bytes each, and output element j (0..15) is
// C[8*(j/4) + 4*(l/32) + j%4][l % 32].
//
// Digit planes live in global memory K-blocked (see SPlanes) with rows and
// inner bytes padded by zero digits, so the GEMM loaders copy 16-byte chunks
// without bounds checks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

typedef int64_t i64;
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kSliceDigits = 4;        // digits per value (planes per operand)
constexpr int kSliceLevel = 6;         // products d_i d_j with i + j <= 6 are kept
constexpr int kSliceKB = 32;           // inner block: bytes per row per block
constexpr int kSliceProdShift = -14;   // a row product is 2^(ea + eb - 14) * sum_l ...
// Most inner indices one int32 level sum may take (see above): at most 4
// digit pairs of |d_i d_j| <= 2^14 per index, so n indices give
// |S_l| <= 2^16 n, below 2^31 for n <= 32767.  Every plan splits its
// contractions so that no accumulation exceeds this depth.
constexpr int kSliceMaxDepth = 32767;

__device__ __forceinline__ v16i mfma_i8(v4i a, v4i b, v16i c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// Scale exponent of a row: the smallest e with maxabs <= 2^e * 127/128 (0 for
// an all-zero row).  Both comparisons are exact in FP64.
__device__ __forceinline__ int row_exponent(double maxabs)
{
    if (!(maxabs > 0.0))
        return 0;
    int e = ilogb(maxabs) + 1;                       // 2^(e-1) <= maxabs < 2^e
    if (maxabs * 128.0 > ldexp(127.0, e))
        e++;
    return e;
}

// The four digits of a, given the row exponent e (|a| <= 2^e * 127/128):
// d[0] is the leading digit.
__device__ __forceinline__ void slice_value(double a, int e, int8_t *d)
{
    int n = (int)rint(ldexp(a, 31 - e));             // |n| <= 127 * 2^24
#pragma unroll
    for (int i = kSliceDigits - 1; i > 0; i--) {
        const int t = ((n + 128) & 255) - 128;
        d[i] = (int8_t)t;
        n = (n - t) >> 8;                            // exact: n - t is a multiple of 256
    }
    d[0] = (int8_t)n;
}

// ---------------------------------------------------------------- planes
// Digit planes in global memory are K-blocked: plane p, row i, inner byte k
// lives at base[p * pstride + (k / 32) * kbstride + i * 32 + k % 32], with
// kbstride = (rows of the array) * 32.  A tile of rows x 32 inner bytes of one
// plane is therefore one contiguous block; rows and inner bytes are padded
// with zero digits, so tile loads need no bounds checks.
struct SPlanes {
    const int8_t *base;   // already offset to the first row of the operand
    i64 pstride;          // bytes between planes
    i64 kbstride;         // bytes between inner blocks
};

// Byte offset of (row, 16-byte half) inside a plane of an LDS stage.  The two
// 16-byte halves of a row swap places on every other group of 8 rows, so the
// 64 lanes of a fragment read (rows r..r+31, half l/32) spread evenly over
// the LDS banks.
__device__ __forceinline__ int slds_off(int row, int half)
{
    return row * kSliceKB + ((half ^ ((row >> 3) & 1)) << 4);
}

// 16 bytes per lane from global memory straight into LDS at dst + 16 * lane
// (dst is the same for the whole wave).  The builtin exists only in the
// device compilation.
__device__ __forceinline__ void global_to_lds16(const int8_t *src, char *dst)
{
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
#endif
}

// ---------------------------------------------------------------- tiles
// Workgroup tile BM x BN; each wave owns 32 x (32 WTN) outputs (WTN MFMA
// tiles side by side), so one A fragment feeds WTN tiles.  Waves (BM/32) x
// (BN/(32 WTN)).  One pipeline stage is one 32-byte inner block of NS planes
// of both operands.
template <int BM, int BN, int NS, int WTN>
struct STileW {
    static constexpr int WROWS = BM / 32, WCOLS = BN / (32 * WTN);
    static constexpr int NWAVE = WROWS * WCOLS;
    static constexpr int NTHR = NWAVE * 64;
    static constexpr int NLEV = kSliceLevel - 1;       // levels 2..kSliceLevel
    static constexpr int TN = WTN;
    static constexpr int A_BYTES = NS * BM * kSliceKB, B_BYTES = NS * BN * kSliceKB;
    static constexpr int STAGE_BYTES = A_BYTES + B_BYTES;
};

template <class TL>
struct SAccW {
    v16i c[TL::TN][TL::NLEV];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int t = 0; t < TL::TN; t++)
#pragma unroll
            for (int l = 0; l < TL::NLEV; l++)
#pragma unroll
                for (int e = 0; e < 16; e++)
                    c[t][l][e] = 0;
    }
};

// ---------------------------------------------------------------- ping-pong GEMM
// acc_l += sum over inner blocks [kb_begin, kb_end) of the kept digit pairs of
// level l, for the 128 x 128 tile of eight waves of 32 x 64 outputs.  The
// waves work in two groups half a stage apart.  Group 0 (waves 0-3, rows
// 0..63) reads a stage's fragments from LDS while group 1 (waves 4-7, rows
// 64..127) multiplies the previous stage's, then the roles swap; every SIMD
// holds one wave of each group, so its matrix core is fed by one group while
// the other waits on LDS.  A workgroup barrier separates the phases.
//
// NBUF LDS stage buffers: the blocks of stage s are copied global -> LDS
// (direct, 16 bytes per lane) in phase 2 (s - NBUF + 1) and must have landed
// by the end of phase 2s - 1, before group 0 reads them in phase 2s.  Stage
// s's buffer is refilled with stage s + NBUF in phase 2s + 2, after the
// barrier that ends group 1's read of stage s (phase 2s + 1).
// s_waitcnt with vmcnt <= n and the other counters unconstrained (gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// LDS of a GEMM pipeline with NB stage buffers.
template <class TL, int NB = 3>
struct SPipe {
    static_assert(NB >= 3 && NB <= 5, "LDS stage buffers");
    static constexpr int NBUF = NB;
    static constexpr int LDS_BYTES = NBUF * TL::STAGE_BYTES;
};

// s_waitcnt vmcnt(n * PER) for a run-time n in [0, NMAX].
template <int PER, int NMAX>
__device__ __forceinline__ void wait_vm_stages(int n)
{
    if (NMAX >= 3 && n >= 3)
        wait_vmcnt<3 * PER>();
    else if (NMAX >= 2 && n == 2)
        wait_vmcnt<2 * PER>();
    else if (NMAX >= 1 && n == 1)
        wait_vmcnt<PER>();
    else
        wait_vmcnt<0>();
}


// A pointer that is the same for every lane of the wave, kept in scalar
// registers.
__device__ __forceinline__ const int8_t *uniform_ptr(const int8_t *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const int8_t *)(((uint64_t)hi << 32) | lo);
}

// Workgroup barrier without the memory fence of __syncthreads(): that fence
// waits for every outstanding global load (vmcnt 0), which would drain the
// copies of later stages.  The waits each phase needs are explicit.  The
// empty asm statements keep memory accesses on their side of it, and the
// scheduling barriers keep every other instruction there too (the compiler
// would otherwise hoist matrix products into the other group's phase).
__device__ __forceinline__ void wg_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

template <class TL, int NS, int NSTAGEBUF = 3>
__device__ __forceinline__ void stile_gemm_pp(const SPlanes &A, const SPlanes &B, int m0, int n0,
                                              int kb_begin, int kb_end, char *lds, SAccW<TL> &acc)
{
    constexpr int BM = TL::WROWS * 32, BN = TL::WCOLS * 32 * TL::TN, WTN = TL::TN;
    constexpr int NBA = NS * (BM / 32), NB = NBA + NS * (BN / 32);
    constexpr int NW = TL::NWAVE, PER = (NB + NW - 1) / NW;
    static_assert(TL::NWAVE == 8 && TL::WROWS == 4 && TL::WCOLS == 2, "two groups of four waves");
    constexpr int NBUF = SPipe<TL, NSTAGEBUF>::NBUF;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int grp = wave >> 2;
    const int nst = kb_end - kb_begin;
    if (nst <= 0)
        return;
    // Block copies: a block is 32 rows x 32 bytes of one plane (1 KB, one
    // wave instruction).  The block's global start and LDS slot are the same
    // for the whole wave; lane l copies row l / 2, half (l & 1) swizzled to
    // the LDS layout of slds_off.
    const uint32_t lane_off = (lane >> 1) * kSliceKB + (((lane & 1) ^ ((lane >> 4) & 1)) << 4);
    const int8_t *ub[PER];
    int loff[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int b = wave + u * NW;
        const int bb = b < NB ? b : 0;
        const bool isA = bb < NBA;
        const int bl = isA ? bb : bb - NBA;
        const int T = isA ? BM : BN;
        const int p = bl / (T / 32), rh = bl % (T / 32);
        const SPlanes &op = isA ? A : B;
        ub[u] = uniform_ptr(op.base + p * op.pstride + (i64)((isA ? m0 : n0) + rh * 32) * kSliceKB);
        loff[u] = (isA ? 0 : TL::A_BYTES) + p * T * kSliceKB + rh * 32 * kSliceKB;
    }
    const i64 akbs = A.kbstride, bkbs = B.kbstride;
    auto issue = [&](int kb, int buf) {
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int b = wave + u * NW;
            if (NB % NW == 0 || b < NB)
                global_to_lds16(ub[u] + (i64)kb * (b < NBA ? akbs : bkbs) + lane_off,
                                lds + buf * TL::STAGE_BYTES + loff[u]);
        }
    };
    const int aoff = slds_off(wr * 32 + (lane & 31), lane >> 5);
    int boff[WTN];
#pragma unroll
    for (int t = 0; t < WTN; t++)
        boff[t] = slds_off((wc * WTN + t) * 32 + (lane & 31), lane >> 5);
    v4i fa[NS], fb[WTN][NS];
    auto read = [&](int st) {
        const char *sa = lds + (st % NBUF) * TL::STAGE_BYTES;
        const char *sb = sa + TL::A_BYTES;
#pragma unroll
        for (int p = 0; p < NS; p++) {
            fa[p] = *(const v4i *)(sa + p * BM * kSliceKB + aoff);
#pragma unroll
            for (int t = 0; t < WTN; t++)
                fb[t][p] = *(const v4i *)(sb + p * BN * kSliceKB + boff[t]);
        }
    };
    // digit pairs (i + 1, j + 1) with i + j + 2 <= kSliceLevel, into level i + j
    auto mult = [&]() {
#pragma unroll
        for (int i = 0; i < NS; i++)
#pragma unroll
            for (int t = 0; t < WTN; t++)
#pragma unroll
                for (int j = 0; j < NS; j++)
                    if (i + j + 2 <= kSliceLevel)
                        acc.c[t][i + j] = mfma_i8(fa[i], fb[t][j], acc.c[t][i + j]);
    };
    // Each group runs its own loop (straight-line bodies, one fragment set
    // each); the workgroup barriers pair up phase by phase:
    //   phase 2s      group 0 reads stage s,       group 1 multiplies stage s - 1
    //   phase 2s + 1  group 0 multiplies stage s,  group 1 reads stage s
    // Both groups issue their copies of stage s in phase 2 (s - NBUF + 1) and
    // wait for them at the end of phase 2s - 1, when the copies of the
    // NBUF - 2 later stages may still be in flight.
    constexpr int AHEAD = NBUF - 1;
    for (int s0 = 0; s0 < AHEAD; s0++)
        if (s0 < nst)
            issue(kb_begin + s0, s0);
    wait_vm_stages<PER, NBUF - 2>(min(nst - 1, AHEAD - 1));
    wg_barrier();
    if (grp == 0) {
#pragma clang loop unroll(disable)
        for (int st = 0; st < nst; st++) {
            if (st + AHEAD < nst)
                issue(kb_begin + st + AHEAD, (st + AHEAD) % NBUF);
            read(st);
            __builtin_amdgcn_s_waitcnt(0xC07F);     // lgkmcnt(0): fragments in registers
            wg_barrier();
            mult();
            // stage st + 1 landed; stages st + 2 .. st + AHEAD may be in flight
            wait_vm_stages<PER, NBUF - 2>(min(nst - st - 2, AHEAD - 1));
            wg_barrier();
        }
    } else {
        if (AHEAD < nst)
            issue(kb_begin + AHEAD, AHEAD % NBUF);
        wg_barrier();
#pragma clang loop unroll(disable)
        for (int st = 0; st < nst; st++) {
            read(st);
            __builtin_amdgcn_s_waitcnt(0xC07F);
            wait_vm_stages<PER, NBUF - 2>(min(nst - st - 2, AHEAD - 1));
            wg_barrier();
            if (st + AHEAD + 1 < nst)
                issue(kb_begin + st + AHEAD + 1, (st + AHEAD + 1) % NBUF);
            mult();
            if (st + 1 < nst)
                wg_barrier();
        }
    }
}

// ---------------------------------------------------------------- four-wave GEMM
// The same product for a workgroup of (BM/32) x (BN/64) = four waves of
// 32 x 64 outputs, small enough for two workgroups per CU: while one
// workgroup waits on LDS, a prologue or its epilogue, the other's products
// keep the matrix cores busy.  All waves read a stage's fragments, multiply,
// then meet at one barrier; NBUF LDS stage buffers, stage s copied
// global -> LDS NBUF - 1 stages ahead.
template <class TL, int NS, int NBUF>
__device__ __forceinline__ void stile_gemm_w4(const SPlanes &A, const SPlanes &B, int m0, int n0,
                                              int kb_begin, int kb_end, char *lds, SAccW<TL> &acc)
{
    static_assert(TL::NWAVE == 4, "four waves");
    constexpr int BM = TL::WROWS * 32, BN = TL::WCOLS * 32 * TL::TN, WTN = TL::TN;
    constexpr int NBA = NS * (BM / 32), NB = NBA + NS * (BN / 32);
    constexpr int NW = TL::NWAVE, PER = (NB + NW - 1) / NW;
    static_assert(NB % NW == 0, "whole blocks per wave");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int nst = kb_end - kb_begin;
    if (nst <= 0)
        return;
    const uint32_t lane_off = (lane >> 1) * kSliceKB + (((lane & 1) ^ ((lane >> 4) & 1)) << 4);
    const int8_t *ub[PER];
    int loff[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int b = wave + u * NW;
        const bool isA = b < NBA;
        const int bl = isA ? b : b - NBA;
        const int T = isA ? BM : BN;
        const int p = bl / (T / 32), rh = bl % (T / 32);
        const SPlanes &op = isA ? A : B;
        ub[u] = uniform_ptr(op.base + p * op.pstride + (i64)((isA ? m0 : n0) + rh * 32) * kSliceKB);
        loff[u] = (isA ? 0 : TL::A_BYTES) + p * T * kSliceKB + rh * 32 * kSliceKB;
    }
    const i64 akbs = A.kbstride, bkbs = B.kbstride;
    auto issue = [&](int kb, int buf) {
#pragma unroll
        for (int u = 0; u < PER; u++)
            global_to_lds16(ub[u] + (i64)kb * (wave + u * NW < NBA ? akbs : bkbs) + lane_off,
                            lds + buf * TL::STAGE_BYTES + loff[u]);
    };
    const int aoff = slds_off(wr * 32 + (lane & 31), lane >> 5);
    int boff[WTN];
#pragma unroll
    for (int t = 0; t < WTN; t++)
        boff[t] = slds_off((wc * WTN + t) * 32 + (lane & 31), lane >> 5);
    constexpr int AHEAD = NBUF - 1;
    for (int s0 = 0; s0 < AHEAD; s0++)
        if (s0 < nst)
            issue(kb_begin + s0, s0);
#pragma clang loop unroll(disable)
    for (int st = 0; st < nst; st++) {
        // stage st landed (this wave's copies), then every wave's (barrier)
        wait_vm_stages<PER, NBUF - 2>(min(nst - st - 1, AHEAD - 1));
        wg_barrier();
        if (st + AHEAD < nst)
            issue(kb_begin + st + AHEAD, (st + AHEAD) % NBUF);
        const char *sa = lds + (st % NBUF) * TL::STAGE_BYTES;
        const char *sb = sa + TL::A_BYTES;
        v4i fa[NS], fb[WTN][NS];
#pragma unroll
        for (int p = 0; p < NS; p++) {
            fa[p] = *(const v4i *)(sa + p * BM * kSliceKB + aoff);
#pragma unroll
            for (int t = 0; t < WTN; t++)
                fb[t][p] = *(const v4i *)(sb + p * BN * kSliceKB + boff[t]);
        }
#pragma unroll
        for (int i = 0; i < NS; i++)
#pragma unroll
            for (int t = 0; t < WTN; t++)
#pragma unroll
                for (int j = 0; j < NS; j++)
                    if (i + j + 2 <= kSliceLevel)
                        acc.c[t][i + j] = mfma_i8(fa[i], fb[t][j], acc.c[t][i + j]);
    }
}

// Output coordinates of element e of tile t of this lane.
template <class TL>
__device__ __forceinline__ void stile_coord_wide(int t, int e, int &row, int &col)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    row = wr * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    col = (wc * TL::TN + t) * 32 + (lane & 31);
}

// FP64 value of output element e of tile t of this lane:
// sum_l S_l 2^(-8 (l - 2)), before the 2^(ea + eb + kSliceProdShift) row and
// column scale.  Every step is exact (power-of-two weights) unless the sum
// needs more than 53 bits.
template <class TL>
__device__ __forceinline__ double combine_levels_wide(const SAccW<TL> &acc, int t, int e)
{
    double v = (double)acc.c[t][TL::NLEV - 1][e];
#pragma unroll
    for (int l = TL::NLEV - 2; l >= 0; l--)
        v = fma(v, 0x1p-8, (double)acc.c[t][l][e]);
    return v;
}

} // namespace jk
