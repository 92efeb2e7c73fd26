// slice_core.hpp -- fixed-point slice products on gfx950 INT8 matrix cores.
//
// Split-precision scheme of the mixed J/K path.  Every FP64 row a[0..n) of an
// operand gets one power-of-two scale 2^e with max|a| < 2^e, and is cut into
// NS signed 7-bit digits (base 2^7, round to nearest, |digit| <= 64):
//     a = 2^(e+1) * sum_{i=1..NS} d_i 2^(-7 i) + rest,  |rest| <= 2^(e - 7 NS)
// so each digit plane holds int8 values.  A product of two rows is
//     sum_k a_k b_k = 2^(ea+eb+2) * sum_{l} 2^(-7 l) * S_l,
//     S_l = sum_{i+j=l} sum_k d_i(a_k) d_j(b_k),
// keeping the pairs with i + j <= NS + 1.  Each S_l is an exact integer: the
// matrix cores multiply int8 digits and accumulate in int32, and
// |S_l| <= 5 * n * 2^12 < 2^31 for n <= kSliceMaxDepth = 104857 inner indices
// per accumulation (enforced by the planner).  The levels are
// combined in FP64 at the end (exact conversions, power-of-two weights), so
// the only approximations are the dropped low digits (relative ~2^-34 for
// NS = 5) and FP64 rounding.
//
// Instruction: V_MFMA_I32_32X32X32_I8 (measured 4.6 POP/s on MI355X, about
// twice the BF16 32x32x16 rate).  Lane layout (measured on the device): lane
// l holds A[row l % 32][k 16*(l/32) .. +15] and B[k 16*(l/32) .. +15][col
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

constexpr int kSliceBits = 7;          // bits per digit
constexpr int kSliceKB = 32;           // inner block: bytes per row per block
// Most inner indices one int32 level sum may take: a level holds at most 5
// digit pairs of |d_i d_j| <= 2^12 per index, so n indices give
// |S_l| <= 5 n 2^12, below 2^31 for n <= 104857.  Every plan splits its
// contractions so that no accumulation exceeds this depth.
constexpr int kSliceMaxDepth = 104857;

__device__ __forceinline__ v16i mfma_i8(v4i a, v4i b, v16i c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// Digits of one value given the row exponent e (max|row| < 2^e):
// d[i] = digit i+1 of a * 2^-e, i < NS.
template <int NS>
__device__ __forceinline__ void slice_value(double a, int e, int8_t *d)
{
    double x = ldexp(a, -e) * 64.0;            // |x| < 64
#pragma unroll
    for (int i = 0; i < NS; i++) {
        const double t = rint(x);
        d[i] = (int8_t)(int)t;
        x = (x - t) * 128.0;                   // |x| <= 64, exact
    }
}

// Exponent with max|row| < 2^e (0 for an all-zero row).
__device__ __forceinline__ int row_exponent(double maxabs)
{
    return maxabs > 0.0 ? ilogb(maxabs) + 1 : 0;
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

// ---------------------------------------------------------------- tile GEMM
// One workgroup: BM x BN output tile, waves (BM/32) x (BN/32), one 32x32
// MFMA tile per wave, NS digit planes per operand, one 32-byte inner block
// per pipeline stage.  LDS stage layout: [plane][row][32 bytes] for A, then
// the same for B.  The two 16-byte halves of a row swap places on every
// other group of 8 rows, so the 64 lanes of a fragment read (rows r..r+31,
// half l/32) spread evenly over the LDS banks.
template <int BM, int BN, int NS>
struct STile {
    static constexpr int WROWS = BM / 32, WCOLS = BN / 32;
    static constexpr int NWAVE = WROWS * WCOLS;
    static constexpr int NTHR = NWAVE * 64;
    static constexpr int NLEV = NS;            // levels 2..NS+1
    static constexpr int A_BYTES = NS * BM * kSliceKB, B_BYTES = NS * BN * kSliceKB;
    static constexpr int STAGE_BYTES = A_BYTES + B_BYTES;
    static constexpr int LDS_BYTES = 2 * STAGE_BYTES;
};

// Byte offset of (row, 16-byte half) inside a plane of an LDS stage.
__device__ __forceinline__ int slds_off(int row, int half)
{
    return row * kSliceKB + ((half ^ ((row >> 3) & 1)) << 4);
}

template <int T, int NS, int NTHR>
struct SLoader {
    // 16-byte chunks per stage: NS planes x T rows x 2 halves
    static constexpr int NCH = NS * T * 2;
    static constexpr int NSTEP = (NCH + NTHR - 1) / NTHR;
    v4i v[NSTEP];

    __device__ __forceinline__ void load(const SPlanes &op, int i0, int kb, int tid)
    {
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            const int c = tid + s * NTHR;
            if (NCH % NTHR == 0 || c < NCH) {
                const int p = c / (T * 2), rr = c % (T * 2);
                v[s] = *(const v4i *)(op.base + p * op.pstride + (i64)kb * op.kbstride +
                                      (i64)i0 * kSliceKB + rr * 16);
            }
        }
    }

    __device__ __forceinline__ void store(char *lds, int tid) const
    {
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            const int c = tid + s * NTHR;
            if (NCH % NTHR == 0 || c < NCH) {
                const int p = c / (T * 2), rr = c % (T * 2);
                *(v4i *)(lds + p * T * kSliceKB + slds_off(rr >> 1, rr & 1)) = v[s];
            }
        }
    }
};

template <class TL>
struct SAcc {
    v16i c[TL::NLEV];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int l = 0; l < TL::NLEV; l++)
#pragma unroll
            for (int e = 0; e < 16; e++)
                c[l][e] = 0;
    }
};

// acc_l += sum over inner blocks [kb_begin, kb_end) of the digit pair
// products with i + j = l + 2 (i, j = 1..NS, i + j <= NS + 1).
//
// Pipeline: the block of stage s is copied global -> registers -> LDS buffer
// s % 2 during stage s - 2, its fragments are read from LDS into registers
// during stage s - 1 (while the MFMAs of stage s - 1 run), and it is
// multiplied in stage s.  One barrier per stage (plus one after the first
// fragment reads); a buffer is refilled only after a barrier that follows
// every read of its previous contents.
template <class TL, int NS>
__device__ __forceinline__ void stile_gemm(const SPlanes &A, const SPlanes &B, int m0, int n0,
                                           int kb_begin, int kb_end, char *lds, SAcc<TL> &acc)
{
    constexpr int BM = TL::WROWS * 32, BN = TL::WCOLS * 32;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    SLoader<BM, NS, TL::NTHR> la;
    SLoader<BN, NS, TL::NTHR> lb;
    const int nst = kb_end - kb_begin;
    if (nst <= 0)
        return;
    la.load(A, m0, kb_begin, tid);
    lb.load(B, n0, kb_begin, tid);
    la.store(lds, tid);
    lb.store(lds + TL::A_BYTES, tid);
    if (nst > 1) {
        la.load(A, m0, kb_begin + 1, tid);
        lb.load(B, n0, kb_begin + 1, tid);
        la.store(lds + TL::STAGE_BYTES, tid);
        lb.store(lds + TL::STAGE_BYTES + TL::A_BYTES, tid);
    }
    __syncthreads();
    const int aoff = slds_off(wr * 32 + (lane & 31), lane >> 5);
    const int boff = slds_off(wc * 32 + (lane & 31), lane >> 5);
    v4i fa[NS], fb[NS];
#pragma unroll
    for (int p = 0; p < NS; p++) {
        fa[p] = *(const v4i *)(lds + p * BM * kSliceKB + aoff);
        fb[p] = *(const v4i *)(lds + TL::A_BYTES + p * BN * kSliceKB + boff);
    }
    // buffer 0 is refilled in the first stage: every wave must have read its
    // stage-0 fragments first
    __syncthreads();
    for (int st = 0; st < nst; st++) {
        const bool more2 = st + 2 < nst;
        if (more2) {
            la.load(A, m0, kb_begin + st + 2, tid);
            lb.load(B, n0, kb_begin + st + 2, tid);
        }
        // fragments of stage st + 1 (on the last stage: a harmless re-read)
        const char *sa = lds + ((st + 1) & 1) * TL::STAGE_BYTES;
        const char *sb = sa + TL::A_BYTES;
        v4i ga[NS], gb[NS];
#pragma unroll
        for (int p = 0; p < NS; p++) {
            ga[p] = *(const v4i *)(sa + p * BM * kSliceKB + aoff);
            gb[p] = *(const v4i *)(sb + p * BN * kSliceKB + boff);
        }
#pragma unroll
        for (int i = 0; i < NS; i++)
#pragma unroll
            for (int j = 0; j < NS - i; j++)          // (i+1) + (j+1) <= NS + 1
                acc.c[i + j] = mfma_i8(fa[i], fb[j], acc.c[i + j]);
#pragma unroll
        for (int p = 0; p < NS; p++) {
            fa[p] = ga[p];
            fb[p] = gb[p];
        }
        if (more2) {
            la.store(lds + (st & 1) * TL::STAGE_BYTES, tid);
            lb.store(lds + (st & 1) * TL::STAGE_BYTES + TL::A_BYTES, tid);
        }
        __syncthreads();
    }
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

// Same product with direct global -> LDS copies (global_load_lds_dwordx4):
// no staging registers.  A wave instruction fills one kilobyte of LDS, lane l
// at byte 16 l (measured), so each lane picks the global 16-byte chunk that
// belongs at its LDS slot of the swizzled layout: the slot (row, half') holds
// the chunk (row, half' ^ swizzle(row)).  A stage is NS planes x (BM + BN) / 32
// such blocks, spread over the waves.  Stage s is copied into buffer s % 2
// at the start of stage s - 2 and waited for at the end of that stage.
template <class TL, int NS, int SCHED = 0>
__device__ __forceinline__ void stile_gemm_direct(const SPlanes &A, const SPlanes &B, int m0, int n0,
                                                  int kb_begin, int kb_end, char *lds,
                                                  SAcc<TL> &acc)
{
    constexpr int BM = TL::WROWS * 32, BN = TL::WCOLS * 32;
    constexpr int NBA = NS * (BM / 32), NB = NBA + NS * (BN / 32);
    constexpr int NW = TL::NWAVE, PER = (NB + NW - 1) / NW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int nst = kb_end - kb_begin;
    if (nst <= 0)
        return;
    const int8_t *gp[PER];
    i64 kbs[PER];
    int loff[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int b = wave + u * NW;
        const int bb = b < NB ? b : 0;
        const bool isA = bb < NBA;
        const int bl = isA ? bb : bb - NBA;
        const int T = isA ? BM : BN;
        const int p = bl / (T / 32), rh = bl % (T / 32);
        const int row = rh * 32 + (lane >> 1);
        const int half = (lane & 1) ^ ((row >> 3) & 1);
        const SPlanes &op = isA ? A : B;
        gp[u] = op.base + p * op.pstride + (i64)((isA ? m0 : n0) + row) * kSliceKB + half * 16;
        kbs[u] = op.kbstride;
        loff[u] = (isA ? 0 : TL::A_BYTES) + p * T * kSliceKB + rh * 32 * kSliceKB;
    }
    auto issue = [&](int kb, int buf) {
#pragma unroll
        for (int u = 0; u < PER; u++)
            if (NB % NW == 0 || wave + u * NW < NB)
                global_to_lds16(gp[u] + (i64)kb * kbs[u], lds + buf * TL::STAGE_BYTES + loff[u]);
    };
    issue(kb_begin, 0);
    if (nst > 1)
        issue(kb_begin + 1, 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int aoff = slds_off(wr * 32 + (lane & 31), lane >> 5);
    const int boff = slds_off(wc * 32 + (lane & 31), lane >> 5);
    v4i fa[NS], fb[NS];
#pragma unroll
    for (int p = 0; p < NS; p++) {
        fa[p] = *(const v4i *)(lds + p * BM * kSliceKB + aoff);
        fb[p] = *(const v4i *)(lds + TL::A_BYTES + p * BN * kSliceKB + boff);
    }
    __syncthreads();     // buffer 0 is refilled in the first stage
    for (int st = 0; st < nst; st++) {
        if (st + 2 < nst)
            issue(kb_begin + st + 2, st & 1);
        const char *sa = lds + ((st + 1) & 1) * TL::STAGE_BYTES;
        const char *sb = sa + TL::A_BYTES;
        v4i ga[NS], gb[NS];
#pragma unroll
        for (int p = 0; p < NS; p++) {
            ga[p] = *(const v4i *)(sa + p * BM * kSliceKB + aoff);
            gb[p] = *(const v4i *)(sb + p * BN * kSliceKB + boff);
        }
#pragma unroll
        for (int i = 0; i < NS; i++)
#pragma unroll
            for (int j = 0; j < NS - i; j++)
                acc.c[i + j] = mfma_i8(fa[i], fb[j], acc.c[i + j]);
        if (SCHED == 1) {
            // next-stage fragment reads first, then the products
            __builtin_amdgcn_sched_group_barrier(0x100, 2 * NS, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, NS * (NS + 1) / 2, 0);
        } else if (SCHED == 2) {
            // one fragment read between consecutive products
#pragma unroll
            for (int q = 0; q < 2 * NS; q++) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, NS * (NS + 1) / 2 - 2 * NS, 0);
        }
#pragma unroll
        for (int p = 0; p < NS; p++) {
            fa[p] = ga[p];
            fb[p] = gb[p];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- wide tiles
// Each wave owns 32 x (32 WTN) outputs (WTN MFMA tiles side by side), so one
// A fragment feeds WTN tiles: fewer LDS bytes per product.  Waves (BM/32) x
// (BN/(32 WTN)).  Direct global -> LDS copies, double-buffered LDS stages,
// fragments read at the start of each stage.
template <int BM, int BN, int NS, int WTN>
struct STileW {
    static constexpr int WROWS = BM / 32, WCOLS = BN / (32 * WTN);
    static constexpr int NWAVE = WROWS * WCOLS;
    static constexpr int NTHR = NWAVE * 64;
    static constexpr int NLEV = NS;
    static constexpr int TN = WTN;
    static constexpr int A_BYTES = NS * BM * kSliceKB, B_BYTES = NS * BN * kSliceKB;
    static constexpr int STAGE_BYTES = A_BYTES + B_BYTES;
    static constexpr int LDS_BYTES = 2 * STAGE_BYTES;
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

template <class TL, int NS>
__device__ __forceinline__ void stile_gemm_wide(const SPlanes &A, const SPlanes &B, int m0, int n0,
                                                int kb_begin, int kb_end, char *lds, SAccW<TL> &acc)
{
    constexpr int BM = TL::WROWS * 32, BN = TL::WCOLS * 32 * TL::TN, WTN = TL::TN;
    constexpr int NBA = NS * (BM / 32), NB = NBA + NS * (BN / 32);
    constexpr int NW = TL::NWAVE, PER = (NB + NW - 1) / NW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int nst = kb_end - kb_begin;
    if (nst <= 0)
        return;
    const int8_t *gp[PER];
    i64 kbs[PER];
    int loff[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int b = wave + u * NW;
        const int bb = b < NB ? b : 0;
        const bool isA = bb < NBA;
        const int bl = isA ? bb : bb - NBA;
        const int T = isA ? BM : BN;
        const int p = bl / (T / 32), rh = bl % (T / 32);
        const int row = rh * 32 + (lane >> 1);
        const int half = (lane & 1) ^ ((row >> 3) & 1);
        const SPlanes &op = isA ? A : B;
        gp[u] = op.base + p * op.pstride + (i64)((isA ? m0 : n0) + row) * kSliceKB + half * 16;
        kbs[u] = op.kbstride;
        loff[u] = (isA ? 0 : TL::A_BYTES) + p * T * kSliceKB + rh * 32 * kSliceKB;
    }
    auto issue = [&](int kb, int buf) {
#pragma unroll
        for (int u = 0; u < PER; u++)
            if (NB % NW == 0 || wave + u * NW < NB)
                global_to_lds16(gp[u] + (i64)kb * kbs[u], lds + buf * TL::STAGE_BYTES + loff[u]);
    };
    const int aoff = slds_off(wr * 32 + (lane & 31), lane >> 5);
    int boff[WTN];
#pragma unroll
    for (int t = 0; t < WTN; t++)
        boff[t] = slds_off((wc * WTN + t) * 32 + (lane & 31), lane >> 5);
    issue(kb_begin, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int st = 0; st < nst; st++) {
        if (st + 1 < nst)
            issue(kb_begin + st + 1, (st + 1) & 1);
        const char *sa = lds + (st & 1) * TL::STAGE_BYTES;
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
                for (int j = 0; j < NS - i; j++)
                    acc.c[t][i + j] = mfma_i8(fa[i], fb[t][j], acc.c[t][i + j]);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// Output coordinates of element e of tile t of this lane (wide tiles).
template <class TL>
__device__ __forceinline__ void stile_coord_wide(int t, int e, int &row, int &col)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    row = wr * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    col = (wc * TL::TN + t) * 32 + (lane & 31);
}

template <class TL>
__device__ __forceinline__ double combine_levels_wide(const SAccW<TL> &acc, int t, int e)
{
    double v = 0.0;
#pragma unroll
    for (int l = TL::NLEV - 1; l >= 0; l--)
        v += ldexp((double)acc.c[t][l][e], -kSliceBits * (l + 2));
    return v;
}

// FP64 value of output element e (0..15) of this lane: sum_l S_l 2^(-7(l+2)),
// before the 2^(ea+eb+2) row/column scale.
template <class TL>
__device__ __forceinline__ double combine_levels(const SAcc<TL> &acc, int e)
{
    double v = 0.0;
#pragma unroll
    for (int l = TL::NLEV - 1; l >= 0; l--)
        v += ldexp((double)acc.c[l][e], -kSliceBits * (l + 2));
    return v;
}

// Output coordinates of element e of this lane inside the workgroup tile.
template <class TL>
__device__ __forceinline__ void stile_coord(int e, int &row, int &col)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    row = wr * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    col = wc * 32 + (lane & 31);
}

} // namespace jk
