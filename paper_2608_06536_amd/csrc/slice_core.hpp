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
// |S_l| <= 5 * n * 2^12 < 2^31 for n <= 100000 inner indices.  The levels are
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
// MFMA tile per wave, NS digit planes per operand.  A stage holds KBS inner
// blocks of 32 bytes.  LDS stage layout: [plane][block][row][32 bytes] for A,
// then the same for B, unpadded: the 16-byte chunks of a stage land in LDS in
// the order they are read from global memory, and a fragment read by 64
// lanes is 2 KB contiguous.  Inner ranges must be multiples of KBS blocks
// (planes are zero-padded to that).
template <int BM, int BN, int NS, int KBS>
struct STile {
    static constexpr int WROWS = BM / 32, WCOLS = BN / 32;
    static constexpr int NWAVE = WROWS * WCOLS;
    static constexpr int NTHR = NWAVE * 64;
    static constexpr int NLEV = NS;            // levels 2..NS+1
    static constexpr int KB = KBS;
    static constexpr int A_BYTES = NS * KBS * BM * kSliceKB, B_BYTES = NS * KBS * BN * kSliceKB;
    static constexpr int STAGE_BYTES = A_BYTES + B_BYTES;
    static constexpr int LDS_BYTES = 2 * STAGE_BYTES;
};

template <int T, int NS, int KBS, int NTHR>
struct SLoader {
    // 16-byte chunks per stage: NS planes x KBS blocks x T rows x 2
    static constexpr int NCH = NS * KBS * T * 2;
    static constexpr int NSTEP = (NCH + NTHR - 1) / NTHR;
    v4i v[NSTEP];

    __device__ __forceinline__ void load(const SPlanes &op, int i0, int kb, int tid)
    {
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            const int c = tid + s * NTHR;
            if (NCH % NTHR == 0 || c < NCH) {
                const int p = c / (KBS * T * 2), rem = c % (KBS * T * 2);
                const int kbl = rem / (T * 2), rr = rem % (T * 2);
                v[s] = *(const v4i *)(op.base + p * op.pstride + (i64)(kb + kbl) * op.kbstride +
                                      (i64)i0 * kSliceKB + rr * 16);
            }
        }
    }

    __device__ __forceinline__ void store(char *lds, int tid) const
    {
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            const int c = tid + s * NTHR;
            if (NCH % NTHR == 0 || c < NCH)
                *(v4i *)(lds + c * 16) = v[s];
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
// kb_end - kb_begin must be a multiple of TL::KB.
template <class TL, int NS>
__device__ __forceinline__ void stile_gemm(const SPlanes &A, const SPlanes &B, int m0, int n0,
                                           int kb_begin, int kb_end, char *lds, SAcc<TL> &acc)
{
    constexpr int BM = TL::WROWS * 32, BN = TL::WCOLS * 32, KBS = TL::KB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    SLoader<BM, NS, KBS, TL::NTHR> la;
    SLoader<BN, NS, KBS, TL::NTHR> lb;
    const int nst = (kb_end - kb_begin) / KBS;
    if (nst <= 0)
        return;
    la.load(A, m0, kb_begin, tid);
    lb.load(B, n0, kb_begin, tid);
    la.store(lds, tid);
    lb.store(lds + TL::A_BYTES, tid);
    __syncthreads();
    const int aoff = (wr * 32 + (lane & 31)) * kSliceKB + 16 * (lane >> 5);
    const int boff = (wc * 32 + (lane & 31)) * kSliceKB + 16 * (lane >> 5);
    for (int st = 0; st < nst; st++) {
        const int cur = st & 1;
        const bool more = st + 1 < nst;
        if (more) {
            la.load(A, m0, kb_begin + (st + 1) * KBS, tid);
            lb.load(B, n0, kb_begin + (st + 1) * KBS, tid);
        }
        const char *sa = lds + cur * TL::STAGE_BYTES;
        const char *sb = sa + TL::A_BYTES;
#pragma unroll
        for (int kbl = 0; kbl < KBS; kbl++) {
            v4i a[NS], b[NS];
#pragma unroll
            for (int p = 0; p < NS; p++) {
                a[p] = *(const v4i *)(sa + (p * KBS + kbl) * BM * kSliceKB + aoff);
                b[p] = *(const v4i *)(sb + (p * KBS + kbl) * BN * kSliceKB + boff);
            }
#pragma unroll
            for (int i = 0; i < NS; i++)
#pragma unroll
                for (int j = 0; j < NS - i; j++)          // (i+1) + (j+1) <= NS + 1
                    acc.c[i + j] = mfma_i8(a[i], b[j], acc.c[i + j]);
        }
        if (more) {
            la.store(lds + (cur ^ 1) * TL::STAGE_BYTES, tid);
            lb.store(lds + (cur ^ 1) * TL::STAGE_BYTES + TL::A_BYTES, tid);
        }
        __syncthreads();
    }
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
