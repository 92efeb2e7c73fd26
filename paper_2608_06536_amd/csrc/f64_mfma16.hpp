// f64_mfma16.hpp -- the second FP64 matrix-core tile engine, on
// V_MFMA_F64_16X16X4_F64.
//
// One instruction is a 16 x 16 x 4 product (2048 flop, four times the work
// of the 4x4x4 form for the same two operand registers), so a wave tile
// needs a quarter of the fragment reads per flop.  Lane mapping (measured on
// the device with one-hot operands):
//   A fragment (16 rows x 4 inner):  lane l holds A[row l & 15][k l >> 4]
//   B fragment (4 inner x 16 cols):  lane l holds B[k l >> 4][col l & 15]
//   output (16 x 16), 4 per lane:    value v of lane l is C[(l >> 4) + 4v][l & 15]
// The instruction reaches its full rate only with the accumulators in
// VGPRs; the compiler picks that form when the launch bounds cap a wave at
// 256 VGPRs or fewer (every kernel using this engine declares a minimum of
// two workgroups of four waves per CU, or more).
//
// Both fragments have the same shape (16 indices x 4 inner), so both operand
// tiles sit in LDS in fragment order: blocks of 64 doubles, [k & 3][i & 15],
// one block per (group of 16 indices, inner step of 4), blocks 68 doubles
// apart.  A fragment read is one contiguous 512-byte read per wave.  The
// 4-double pad keeps the loader's writes free of bank conflicts.
//
// Operands are read with buffer loads: a 128-bit resource (base, size in
// bytes) in scalar registers, a per-lane byte offset computed once per tile,
// and the stage's advance along the inner index as a scalar offset, so a
// stage's loads cost no vector address arithmetic.  Each lane loads a run of
// consecutive doubles along the operand's contiguous index (four k, or two
// i; see BufLoader).  Indices are clamped to the operand once per tile; inner indices
// past the end are zeroed in the last stage only.  A read past the
// resource's size returns zero (the hardware's range check).
#pragma once
#include "f64_core.hpp"

namespace jk {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4v mfma16(double a, double b, d4v c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A value that is the same in every lane of the wave (it depends on the
// workgroup index and kernel arguments only), moved to scalar registers.  A
// buffer resource must be built from scalar values: where the compiler cannot
// prove a base or size uniform, it wraps every load in a per-lane loop.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ const char *wave_uniform(const char *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (const char *)(((unsigned long long)hi << 32) | lo);
}

// Operand element (i, k), i the row of A or the column of B, k the inner
// index, valid for i < ni, k < nk:
//   BufKC: at p[i ld + k]  (k contiguous)
//   BufIC: at p[k ld + i]  (i contiguous)
// Host code must keep the operand's extent below 4 GiB (buf_extent_ok).
// In a segmented product every segment gets a resource of its own.
struct BufKC {
    static constexpr bool kContig = true;
    const double *p;
    i64 ld;
    int ni, nk;
    __device__ __forceinline__ i64 extent() const { return ((i64)(ni - 1) * ld + nk) * 8; }
};
struct BufIC {
    static constexpr bool kContig = false;
    const double *p;
    i64 ld;
    int ni, nk;
    __device__ __forceinline__ i64 extent() const { return ((i64)(nk - 1) * ld + ni) * 8; }
};
__host__ __device__ inline bool buf_extent_ok(i64 elements) { return elements * 8 < (1LL << 32); }

template <int BM_, int BN_, int WM_, int WN_, int BK_>
struct Tile16 {
    static constexpr bool kMfma16 = true;
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, BK = BK_;
    static constexpr int WROWS = BM / WM, WCOLS = BN / WN;
    static constexpr int NWAVE = WROWS * WCOLS;
    static constexpr int NTHR = NWAVE * 64;
    static constexpr int MA = WM / 16, NB = WN / 16, NSUB = BK / 4;
    static constexpr int BLK = 68;                          // doubles per fragment block
    static constexpr int A_DOUBLES = (BM / 16) * NSUB * BLK, B_DOUBLES = (BN / 16) * NSUB * BLK;
    static constexpr int STAGE = A_DOUBLES + B_DOUBLES;
    static constexpr int LDS_DOUBLES = 2 * STAGE;
    static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 16 == 0, "tile16");
    static_assert(BK % 4 == 0 && (BM * BK / 4) % NTHR == 0 && (BN * BK / 4) % NTHR == 0, "tile16");
};

template <class TL>
struct Acc16 {
    d4v c[TL::MA][TL::NB];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < TL::MA; i++)
#pragma unroll
            for (int j = 0; j < TL::NB; j++)
                c[i][j] = (d4v){0.0, 0.0, 0.0, 0.0};
    }
};

// fragment-order slot of element (i, k) within a stage's operand tile
template <int NSUB>
__device__ __forceinline__ int frag_slot(int i, int k)
{
    return ((i >> 4) * NSUB + (k >> 2)) * 68 + 16 * (k & 3) + (i & 15);
}

// Moves a T x BK operand tile in groups of consecutive elements along the
// contiguous index, group g = tid + s NTHR:
//   BufKC: four consecutive k of one row i (two 16-byte loads).  A lane's
//     four values go to four rows of a fragment block, 128 bytes apart.
//   BufIC: two consecutive i of one inner index k (one 16-byte load).  The
//     16 lanes that one LDS write cycle serves then cover 256 consecutive
//     bytes of two fragment blocks, one bank each; groups of four i put
//     lanes 8 apart on the same banks (the blocks of one k are 272 doubles
//     apart).
template <int T, int BK, int NTHR, class Op>
struct BufLoader {
    static constexpr int G = Op::kContig ? 4 : 2;
    static constexpr int NGRP = T * BK / G, NS = NGRP / NTHR, NSUB = BK / 4;
    static_assert(NGRP % NTHR == 0, "operand tile and thread count");
    const char *base;      // segment 0
    int nbytes;            // extent of one segment (bit pattern of an unsigned)
    unsigned voff[NS];     // byte offset of the group at inner index 0 of the tile
    double raw[NS][G];

    // local (i, k) of the first element of group s
    __device__ __forceinline__ static void local(int g, int &li, int &lk)
    {
        if (Op::kContig) {
            li = g / (BK / 4);
            lk = (g % (BK / 4)) * 4;
        } else {
            lk = g / (T / 2);
            li = (g % (T / 2)) * 2;
        }
    }

    // Per tile: i0 = first index of the tile, kb = first inner index.
    __device__ __forceinline__ void init(const Op &op, int i0, int kb, int tid)
    {
        base = wave_uniform((const char *)op.p);
        nbytes = wave_uniform((int)op.extent());
#pragma unroll
        for (int s = 0; s < NS; s++) {
            int li, lk;
            local(tid + s * NTHR, li, lk);
            int i = i0 + li;
            if (Op::kContig)
                i = i < op.ni ? i : op.ni - 1;       // rows past the end: clamped
            voff[s] = Op::kContig ? (unsigned)(((i64)i * op.ld + kb + lk) * 8)
                                  : (unsigned)(((i64)(kb + lk) * op.ld + i) * 8);
        }
    }

    // Loads the stage at inner index kk (from the tile's first) of segment
    // seg, segments seg_bytes apart.
    __device__ __forceinline__ void load(const Op &op, int seg, int kk, i64 seg_bytes, int = 0)
    {
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(base + seg * seg_bytes), (short)0, nbytes, 0x00020000);
        const unsigned soff = (unsigned)(Op::kContig ? (i64)kk * 8 : (i64)kk * op.ld * 8);
#pragma unroll
        for (int s = 0; s < NS; s++) {
            const u4v lo = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[s], soff, 0);
            const double2 a = __builtin_bit_cast(double2, lo);
            raw[s][0] = a.x;
            raw[s][1] = a.y;
            if constexpr (G == 4) {
                const u4v hi = __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[s] + 16, soff, 0);
                const double2 b = __builtin_bit_cast(double2, hi);
                raw[s][2] = b.x;
                raw[s][3] = b.y;
            }
        }
    }

    // Writes the stage into LDS.  With MASK, elements at local inner index
    // kleft or beyond (possible in a tile's last stage only) are then
    // overwritten with zero by the thread that wrote them, in a branch taken
    // only by such a stage, so the other stages carry no selects.
    template <bool MASK>
    __device__ __forceinline__ void store(double *lds, int tid, int kleft) const
    {
#pragma unroll
        for (int s = 0; s < NS; s++) {
            int li, lk;
            local(tid + s * NTHR, li, lk);
#pragma unroll
            for (int e = 0; e < G; e++) {
                const int i = Op::kContig ? li : li + e, k = Op::kContig ? lk + e : lk;
                lds[frag_slot<NSUB>(i, k)] = raw[s][e];
            }
        }
        if (MASK && kleft < BK) {
#pragma unroll
            for (int s = 0; s < NS; s++) {
                int li, lk;
                local(tid + s * NTHR, li, lk);
#pragma unroll
                for (int e = 0; e < G; e++) {
                    const int i = Op::kContig ? li : li + e, k = Op::kContig ? lk + e : lk;
                    if (k >= kleft)
                        lds[frag_slot<NSUB>(i, k)] = 0.0;
                }
            }
        }
    }
};

// A symmetric nao x nao slab stored as its upper triangle, row by row:
// element (a, b), a <= b, at p[a (2 nao - a + 1) / 2 + b - a].  As an
// operand: element (i, k), i the row of A, k the inner index.
struct BufPackedSym {
    const double *p;
    int nao;
    __device__ __forceinline__ i64 extent() const { return (i64)nao * (nao + 1) / 2 * 8; }
};
__device__ __forceinline__ int pk_row16(int a, int nao) { return (int)((i64)a * (2 * nao - a + 1) / 2); }

// Loader of a packed symmetric operand.  Each stage takes one of three
// forms, the same for every thread (it depends on the tile's rows and the
// stage's inner range only):
//   above the diagonal (k >= i throughout): row i of the packed storage is
//     contiguous in k; groups of 4 consecutive k, offsets fixed per tile plus
//     a scalar advance;
//   below it (k <= i throughout): element (i, k) = (k, i) is packed row k,
//     contiguous in i; groups of 2 consecutive i, one row offset per group
//     (pairs keep the LDS writes' bank conflicts low, as for BufIC);
//   on the diagonal: each element's own offset.
// Indices are clamped to the slab.  Inner indices past nao read data of the
// next packed row (finite) or zero past the slab; the caller's other operand
// must read zero there (no mask).
template <int T, int BK, int NTHR>
struct PackedLoader16 {
    static constexpr int NGRP = T * BK / 4, NS = NGRP / NTHR, NSUB = BK / 4;
    static_assert(NGRP % NTHR == 0, "packed loader");
    const char *base;
    int nbytes, nao, i0, kb;
    int mode, k0;          // of the stage held in raw: 0 above, 1 below, 2 diagonal
    unsigned rowoff[NS];   // above: byte offset of (row, inner 0) for group s, kContig mapping
    double raw[NS][4];

    __device__ __forceinline__ static void local_k(int g, int &li, int &lk)
    {
        li = g / (BK / 4);
        lk = (g % (BK / 4)) * 4;
    }
    __device__ __forceinline__ static void local_i(int g, int &li, int &lk)
    {
        lk = g / (T / 2);
        li = (g % (T / 2)) * 2;
    }

    __device__ __forceinline__ void init(const BufPackedSym &op, int i0_, int kb_, int tid)
    {
        base = wave_uniform((const char *)op.p);
        nbytes = wave_uniform((int)op.extent());
        nao = op.nao;
        i0 = i0_;
        kb = kb_;
#pragma unroll
        for (int s = 0; s < NS; s++) {
            int li, lk;
            local_k(tid + s * NTHR, li, lk);
            int i = i0 + li;
            i = i < nao ? i : nao - 1;
            rowoff[s] = (unsigned)(((i64)pk_row16(i, nao) - i + kb + lk) * 8);
        }
    }

    __device__ __forceinline__ void load(const BufPackedSym &, int, int kk, i64, int tid)
    {
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, nbytes, 0x00020000);
        k0 = kb + kk;
        mode = (k0 >= i0 + T - 1) ? 0 : (k0 + BK - 1 <= i0) ? 1 : 2;
        if (mode == 0) {
            const unsigned soff = (unsigned)kk * 8;
#pragma unroll
            for (int s = 0; s < NS; s++) {
                const u4v lo = __builtin_amdgcn_raw_buffer_load_b128(rsrc, rowoff[s], soff, 0);
                const u4v hi = __builtin_amdgcn_raw_buffer_load_b128(rsrc, rowoff[s] + 16, soff, 0);
                const double2 a = __builtin_bit_cast(double2, lo), b = __builtin_bit_cast(double2, hi);
                raw[s][0] = a.x;
                raw[s][1] = a.y;
                raw[s][2] = b.x;
                raw[s][3] = b.y;
            }
        } else if (mode == 1) {
            // 2 NS pairs: pair u in raw[u / 2][2 (u % 2) ..]
#pragma unroll
            for (int u = 0; u < 2 * NS; u++) {
                int li, lk;
                local_i(tid + u * NTHR, li, lk);
                const int k = k0 + lk;                       // < nao below the diagonal
                const unsigned off = (unsigned)(((i64)pk_row16(k, nao) - k + i0 + li) * 8);
                const u4v lo = __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0);
                const double2 a = __builtin_bit_cast(double2, lo);
                raw[u / 2][2 * (u % 2)] = a.x;
                raw[u / 2][2 * (u % 2) + 1] = a.y;
            }
        } else {
#pragma unroll
            for (int s = 0; s < NS; s++) {
                int li, lk;
                local_k(tid + s * NTHR, li, lk);
                int i = i0 + li;
                i = i < nao ? i : nao - 1;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int k = k0 + lk + e;
                    k = k < nao ? k : nao - 1;
                    const int a = i < k ? i : k, b = i < k ? k : i;
                    const unsigned off = (unsigned)(((i64)pk_row16(a, nao) + b - a) * 8);
                    raw[s][e] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0));
                }
            }
        }
    }

    template <bool MASK>
    __device__ __forceinline__ void store(double *lds, int tid, int) const
    {
        static_assert(!MASK, "a packed operand is used unmasked");
        if (mode == 1) {
#pragma unroll
            for (int u = 0; u < 2 * NS; u++) {
                int li, lk;
                local_i(tid + u * NTHR, li, lk);
                lds[frag_slot<NSUB>(li, lk)] = raw[u / 2][2 * (u % 2)];
                lds[frag_slot<NSUB>(li + 1, lk)] = raw[u / 2][2 * (u % 2) + 1];
            }
        } else {
#pragma unroll
            for (int s = 0; s < NS; s++) {
                int li, lk;
                local_k(tid + s * NTHR, li, lk);
#pragma unroll
                for (int e = 0; e < 4; e++)
                    lds[frag_slot<NSUB>(li, lk + e)] = raw[s][e];
            }
        }
    }
};

// The loader of each operand type.
template <int T, int BK, int NTHR, class Op>
struct LoaderOf {
    typedef BufLoader<T, BK, NTHR, Op> type;
};
template <int T, int BK, int NTHR>
struct LoaderOf<T, BK, NTHR, BufPackedSym> {
    typedef PackedLoader16<T, BK, NTHR> type;
};

// acc += sum over segments g < nseg of sum over k in [k_begin, k_begin +
// kdepth) of A_g(m0 + i, k) * B_g(n0 + j, k), where A_g is A with its base
// moved by g segA elements (B_g likewise).  The stages of all segments form
// one pipeline.
//
// Pipeline: two LDS stages and two register sets of global loads.  While
// stage kt is multiplied out of LDS, the loads of stage kt + 2 are in flight
// into one register set and stage kt + 1, loaded one stage earlier, is
// written from the other set into the second LDS stage; one barrier per
// stage.  A load therefore has a full stage of products to arrive before
// its data are written to LDS (measured: 63.0 -> 65.1 TF on the
// half-transform, against the compiler's own order, which sank the loads
// below the products).
template <class TL, class OA, class OB, bool MASK>
struct Gemm16 {
    static constexpr int BK = TL::BK, NSUB = TL::NSUB;
    typedef typename LoaderOf<TL::BM, BK, TL::NTHR, OA>::type LA;
    typedef typename LoaderOf<TL::BN, BK, TL::NTHR, OB>::type LB;

    struct Seq {             // stage kt -> (segment, inner offset)
        int nks, kdepth;
        i64 sega, segb;      // bytes
        __device__ __forceinline__ void at(int kt, int &g, int &kk) const
        {
            g = kt / nks;
            kk = (kt - g * nks) * BK;
        }
    };

    __device__ static __forceinline__ void products(const double *lds, int cur, int fa, int fb,
                                                    Acc16<TL> &acc)
    {
        const double *pa = lds + cur * TL::STAGE + fa;
        const double *pb = lds + cur * TL::STAGE + fb;
#pragma unroll
        for (int s = 0; s < NSUB; s++) {
            double a[TL::MA], b[TL::NB];
#pragma unroll
            for (int i = 0; i < TL::MA; i++)
                a[i] = pa[(i * NSUB + s) * 68];
#pragma unroll
            for (int j = 0; j < TL::NB; j++)
                b[j] = pb[(j * NSUB + s) * 68];
#pragma unroll
            for (int i = 0; i < TL::MA; i++)
#pragma unroll
                for (int j = 0; j < TL::NB; j++)
                    acc.c[i][j] = mfma16(a[i], b[j], acc.c[i][j]);
        }
    }

    // One stage: loads of stage kt + 2 into (la_n, lb_n); stage kt + 1,
    // loaded one stage earlier, from (la_s, lb_s) into the LDS buffer the
    // previous stage read (free since that stage's barrier); products of
    // stage kt; barrier.
    __device__ static __forceinline__ void stage(const OA &A, const OB &B, const Seq &q, int kt,
                                                 int nk, double *lds, int fa, int fb, int tid,
                                                 LA &la_n, LB &lb_n, const LA &la_s,
                                                 const LB &lb_s, Acc16<TL> &acc)
    {
        {
            // Issued first and on every stage (past the end: the last stage
            // again, never written to LDS).  The scheduling barrier keeps the
            // compiler from sinking them below the products, and the fixed
            // count per stage lets the wait before the LDS writes below cover
            // the previous stage's loads only, so a load has a whole stage of
            // products to arrive.
            int g, kk;
            q.at(kt + 2 < nk ? kt + 2 : nk - 1, g, kk);
            la_n.load(A, g, kk, q.sega, tid);
            lb_n.load(B, g, kk, q.segb, tid);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (kt + 1 < nk) {
            int g, kk;
            q.at(kt + 1, g, kk);
            const int kleft = q.kdepth - kk;
            la_s.template store<MASK>(lds + ((kt + 1) & 1) * TL::STAGE, tid, kleft);
            lb_s.template store<MASK>(lds + ((kt + 1) & 1) * TL::STAGE + TL::A_DOUBLES, tid, kleft);
        }
        products(lds, kt & 1, fa, fb, acc);
        __syncthreads();
    }

    __device__ static __forceinline__ void run(const OA &A, const OB &B, int m0, int n0,
                                               int k_begin, int kdepth, int nseg, i64 segA,
                                               i64 segB, double *lds, Acc16<TL> &acc)
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
        Seq q;
        q.nks = (kdepth + BK - 1) / BK;
        q.kdepth = kdepth;
        q.sega = segA * 8;
        q.segb = segB * 8;
        const int nk = q.nks * nseg;
        if (nk <= 0)
            return;
        LA la0, la1;
        LB lb0, lb1;
        la0.init(A, m0, k_begin, tid);
        lb0.init(B, n0, k_begin, tid);
        la1 = la0;
        lb1 = lb0;
        la0.load(A, 0, 0, q.sega, tid);
        lb0.load(B, 0, 0, q.segb, tid);
        if (nk > 1) {
            int g, kk;
            q.at(1, g, kk);
            la1.load(A, g, kk, q.sega, tid);
            lb1.load(B, g, kk, q.segb, tid);
        }
        la0.template store<MASK>(lds, tid, kdepth);
        lb0.template store<MASK>(lds + TL::A_DOUBLES, tid, kdepth);
        __syncthreads();
        const int fa = wr * TL::MA * NSUB * 68 + lane;
        const int fb = TL::A_DOUBLES + wc * TL::NB * NSUB * 68 + lane;
        // register set of stage s: s & 1 (set 0 holds stages 0, 2, 4, ...)
        int kt = 0;
        for (; kt + 1 < nk; kt += 2) {
            stage(A, B, q, kt, nk, lds, fa, fb, tid, la0, lb0, la1, lb1, acc);
            stage(A, B, q, kt + 1, nk, lds, fa, fb, tid, la1, lb1, la0, lb0, acc);
        }
        if (kt < nk)
            products(lds, kt & 1, fa, fb, acc);
    }
};

// acc += sum over k in [k_begin, k_end) of A(m0 + i, k) * B(n0 + j, k).
// MASK false: inner indices past k_end are not zeroed.  Exact only when
// the other operand reads zero there (for instance through the range check
// at the end of its resource) and these elements are finite.
template <class TL, bool MASK = true, class OA, class OB>
__device__ __forceinline__ void tile_gemm16(const OA &A, const OB &B, int m0, int n0, int k_begin,
                                            int k_end, double *lds, Acc16<TL> &acc)
{
    Gemm16<TL, OA, OB, MASK>::run(A, B, m0, n0, k_begin, k_end - k_begin, 1, 0, 0, lds, acc);
}

// acc += sum over g < nseg of the product over k in [0, kdepth) of A_g and
// B_g (bases moved by g segA and g segB elements).
template <class TL, class OA, class OB>
__device__ __forceinline__ void tile_gemm16_seg(const OA &A, const OB &B, i64 segA, i64 segB,
                                                int nseg, int m0, int n0, int kdepth, double *lds,
                                                Acc16<TL> &acc)
{
    Gemm16<TL, OA, OB, true>::run(A, B, m0, n0, 0, kdepth, nseg, segA, segB, lds, acc);
}

// Calls f(row, col, value) for every output element this lane holds: value v
// of accumulator (i, j) is element (m0 + wr WM + 16 i + (lane >> 4) + 4 v,
// n0 + wc WN + 16 j + (lane & 15)).
template <class TL, class F>
__device__ __forceinline__ void tile_foreach16(const Acc16<TL> &acc, int m0, int n0, F &&f)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int rb = m0 + wr * TL::WM + (lane >> 4);
    const int cb = n0 + wc * TL::WN + (lane & 15);
#pragma unroll
    for (int i = 0; i < TL::MA; i++)
#pragma unroll
        for (int j = 0; j < TL::NB; j++)
#pragma unroll
            for (int v = 0; v < 4; v++)
                f(rb + 16 * i + 4 * v, cb + 16 * j, acc.c[i][j][v]);
}

// out[m ld + n] = (accumulate ? out[m ld + n] : 0) + scale * value for every
// output element (m, n) this lane holds with m < mlim and n < nlim.  The four
// elements of an accumulator are read together before any of them is
// written, so that the reads' latencies overlap instead of following each
// other.
template <class TL>
__device__ __forceinline__ void tile_update16(const Acc16<TL> &acc, int m0, int n0,
                                              double *__restrict__ out, i64 ld, int mlim, int nlim,
                                              int accumulate, double scale)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int rb = m0 + wr * TL::WM + (lane >> 4);
    const int cb = n0 + wc * TL::WN + (lane & 15);
#pragma unroll
    for (int i = 0; i < TL::MA; i++)
#pragma unroll
        for (int j = 0; j < TL::NB; j++) {
            const int n = cb + 16 * j;
            double old[4];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int m = rb + 16 * i + 4 * v;
                old[v] = (accumulate && m < mlim && n < nlim) ? out[(i64)m * ld + n] : 0.0;
            }
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int m = rb + 16 * i + 4 * v;
                if (m < mlim && n < nlim)
                    out[(i64)m * ld + n] =
                        accumulate ? old[v] + scale * acc.c[i][j][v] : scale * acc.c[i][j][v];
            }
        }
}

} // namespace jk
