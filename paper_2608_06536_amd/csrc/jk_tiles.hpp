// jk_tiles.hpp -- one workgroup's share of each FP64 build phase.
//
// Every phase of the build is a set of independent tiles; these device
// functions compute one tile.  The single-problem kernels (jk_fp64.hip) run
// tile blockIdx.x of one problem; the batched kernels (jk_batched.hip) map
// blockIdx.x to (problem, tile) through a table and run the same function, so
// a member of a batch is computed exactly as it would be alone.
//
// Phases (Sec. 2.3, Eq. (4), half-transform form K = B_V^T B_U):
//   pack          Cc[n][c]       = [C_L | C_R] as one nao x 2R matrix
//   density       D_k            = C_Lk C_Rk^T
//   project       part[p][Q][k]  = sum over a block of positions of B^Q . A_k
//   reduce        g[k][Q]        = sum of the partials in fixed order
//   coulomb       J_k            = sum_Q gamma_kQ B^Q
//   half-transform X^Q, Y^Q      = B^Q [C_L | C_R]            (per Q-chunk)
//   exchange      K_k           += sum_{Q in chunk} X^Q_k (Y^Q_k)^T
//   sum splits    K              = sum of the split partials in fixed order
// Chunk workspace: X_ws[k][m][ql*r + i], Y_ws likewise, so each exchange
// operand row is contiguous over the chunk's inner index (Q, i).
#pragma once
#include "f64_core.hpp"
#include "f64_mfma16.hpp"

namespace jk {

// Tile shapes (chosen by measurement on MI355X): the half-transform uses
// 128 x 64 workgroup tiles of four 64 x 32 wave tiles (two workgroups per
// CU); the exchange product 128 x 64 tiles of eight 64 x 16 wave tiles (four
// waves per SIMD); the projection 256 Q-rows x 8 densities; the density
// 64 x 64.  Element-wise phases take 1024 elements per tile.
constexpr int kHtM = 128, kHtN = 64;
constexpr int kExM = 128, kExN = 64;
constexpr int kProjRows = 256;
constexpr int kElemTile = 1024;
typedef Tile<kHtM, kHtN, 64, 32, 16> TileHalf;
typedef Tile<kExM, kExN, 64, 16, 16> TileExch;
typedef Tile<kProjRows, 8, 64, 8, 16> TileProject;
typedef Tile<kProjRows, 16, 64, 16, 16> TileProject16;
typedef Tile<64, 64, 32, 32, 16> TileDensity;
// The half-transform's second tile shape (a plan choice, jk_tune.h): 64 x 64,
// four workgroups per CU; wins at small nao where 128-row tiles waste rows.
typedef Tile<64, 64, 32, 32, 16> TileHalf64;
// The default half-transform tile (jk_tune.h tile 4): 128 x 64 on the 16 x 16 x 4
// engine, four 64 x 32 wave tiles, over stacked slabs.
typedef Tile16<128, 64, 64, 32, 16> TileHalf16;

__host__ __device__ inline int cdiv_i(i64 a, i64 b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ packed slabs
// A symmetric slab stored as its upper triangle, row by row: element (m, n),
// m <= n, at pk_row(m) + (n - m), pk_row(m) = m nao - m (m - 1) / 2;
// nao (nao + 1) / 2 doubles per slab.
__host__ __device__ inline i64 pk_size(int nao) { return (i64)nao * (nao + 1) / 2; }
__host__ __device__ inline i64 pk_row(int m, int nao) { return (i64)m * (2 * (i64)nao - m + 1) / 2; }
__host__ __device__ inline i64 pk_index(int m, int n, int nao)
{
    const int a = m < n ? m : n, b = m < n ? n : m;
    return pk_row(a, nao) + (b - a);
}

// element (i, k) of a packed symmetric nao x nao slab, as an A operand of the
// tile engine (both indices clamped for the load, zero outside).  Measured:
// the row-major thread mapping already coalesces below the diagonal (sixteen
// consecutive rows of one column are 128 contiguous bytes), and a per-stage
// column mapping there was no faster.
struct OpPackedSym {
    static constexpr bool kContig = true;
    static constexpr int NRAW = 1;
    const double *p;
    int nao;
    __device__ __forceinline__ void fetch(int i, int k, double *raw) const
    {
        const int ic = i < nao ? i : nao - 1, kc = k < nao ? k : nao - 1;
        raw[0] = p[pk_index(ic, kc, nao)];
    }
    __device__ __forceinline__ double finish(int i, int k, const double *raw) const
    {
        return (i < nao && k < nao) ? raw[0] : 0.0;
    }
};


// ------------------------------------------------------------------ tile counts
__host__ __device__ inline int pack_tiles(int nao, int nd, int r)
{
    return cdiv_i((i64)nao * 2 * nd * r, kElemTile);
}
__host__ __device__ inline int density_tiles(int nao, int nd)
{
    const int nt = cdiv_i(nao, 64);
    return nd * nt * nt;
}
__host__ __device__ inline int project_tiles(int naux, int nd, int npb)
{
    return cdiv_i(naux, kProjRows) * cdiv_i(nd, 8) * npb;
}
__host__ __device__ inline int reduce_tiles(int naux, int nd) { return cdiv_i((i64)naux * (cdiv_i(nd, 8) * 8), 64); }
__host__ __device__ inline int coulomb_tiles(int nd, i64 npos) { return cdiv_i(nd, 8) * cdiv_i(npos, 512); }
__host__ __device__ inline int ht_tiles(int nao, int nd, int r, int nq)
{
    return nq * cdiv_i(nao, kHtM) * cdiv_i(2 * (i64)nd * r, kHtN);
}
__host__ __device__ inline int ht64_tiles(int nao, int nd, int r, int nq)
{
    return nq * cdiv_i(nao, 64) * cdiv_i(2 * (i64)nd * r, 64);
}
// ncol = 2R (X and Y) or R (X only, symmetric densities)
__host__ __device__ inline int ht_tiles_cols(int nao, int ncol, int nq)
{
    return nq * cdiv_i(nao, kHtM) * cdiv_i(ncol, kHtN);
}
__host__ __device__ inline int ex_tiles(int nao, int nd, int nsplit)
{
    return nsplit * nd * cdiv_i(nao, kExM) * cdiv_i(nao, kExN);
}

// Symmetric exchange (C_L = C_R, K = sum X X^T): only the tiles that reach
// the upper triangle n >= m, row tile mb from column tile (mb kExM) / kExN on.
__host__ __device__ inline int ex_tri_first(int mb) { return (mb * kExM) / kExN; }
__host__ __device__ inline int ex_tri_tiles(int nao)
{
    const int nmt = cdiv_i(nao, kExM), nnt = cdiv_i(nao, kExN);
    int n = 0;
    for (int mb = 0; mb < nmt; mb++) {
        const int f = ex_tri_first(mb);
        n += f < nnt ? nnt - f : 0;
    }
    return n;
}
__host__ __device__ inline void ex_tri_coords(int t, int nao, int &mb, int &nb)
{
    const int nmt = cdiv_i(nao, kExM), nnt = cdiv_i(nao, kExN);
    for (mb = 0; mb < nmt; mb++) {
        const int f = ex_tri_first(mb);
        const int cnt = f < nnt ? nnt - f : 0;
        if (t < cnt) {
            nb = f + t;
            return;
        }
        t -= cnt;
    }
    mb = nmt - 1;
    nb = nnt - 1;
}
__host__ __device__ inline int sum_tiles(i64 n) { return cdiv_i(n, kElemTile); }

// Kk[m][n] = Kk[n][m] for m > n in lower-triangle block b of 32 x 32 (blocks
// (bi, bj), bi >= bj, numbered row by row): fills the lower triangle from the
// upper one through an LDS transpose.  256 threads; t is 32 x 33 doubles.
__device__ __forceinline__ void mirror_tile(double *__restrict__ Kk, int nao, int b,
                                            double (*t)[33])
{
    int bi = 0;
    while (b > bi) {
        b -= bi + 1;
        bi++;
    }
    const int bj = b;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int y = ty; y < 32; y += 8) {
        const int row = bj * 32 + y, col = bi * 32 + tx;       // upper source
        if (row < nao && col < nao)
            t[y][tx] = Kk[(i64)row * nao + col];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int m = bi * 32 + y, n = bj * 32 + tx;           // lower target
        if (m < nao && n < nao && m > n)
            Kk[(i64)m * nao + n] = t[tx][y];
    }
    __syncthreads();
}

__host__ __device__ inline int mirror_blocks(int nao)
{
    const int nb = cdiv_i(nao, 32);
    return nb * (nb + 1) / 2;
}

// ------------------------------------------------------------------ pack
__device__ inline void pack_tile(const double *__restrict__ CL, const double *__restrict__ CR,
                                 double *__restrict__ Cc, int nao, int nd, int r, int tile)
{
    const int R = nd * r, R2 = 2 * R;
    const i64 total = (i64)nao * R2;
    for (int u = 0; u < kElemTile / 256; u++) {
        const i64 e = (i64)tile * kElemTile + u * 256 + threadIdx.x;
        if (e < total) {
            const int n = (int)(e / R2), c = (int)(e % R2);
            const double *src = c < R ? CL : CR;
            const int cc = c < R ? c : c - R;
            const int k = cc / r, i = cc % r;
            Cc[e] = src[((i64)k * nao + n) * r + i];
        }
    }
}

// ------------------------------------------------------------------ density
// D_k[m][n] = sum_i CL[k][m][i] CR[k][n][i]
__device__ inline void density_tile(const double *__restrict__ CL, const double *__restrict__ CR,
                                    double *__restrict__ D, int nao, int r, int tile, double *lds)
{
    typedef TileDensity TL;
    const int nt = cdiv_i(nao, 64);
    const int k = tile / (nt * nt), rem = tile % (nt * nt);
    const int mb = rem / nt, nb = rem % nt;
    OpKC a{CL + (i64)k * nao * r, r, nao, r};
    OpKC b{CR + (i64)k * nao * r, r, nao, r};
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, mb * 64, nb * 64, 0, r, lds, acc);
    double *Dk = D + (i64)k * nao * nao;
    tile_foreach(acc, mb * 64, nb * 64, [&](int m, int n, double v) {
        if (m < nao && n < nao)
            Dk[(i64)m * nao + n] = v;
    });
}

// ------------------------------------------------------------------ project
// part[pb][Q][kg*8 + kk] = sum_{p in block pb} B[Q][p] * A[kg*8 + kk][p]:
// a product with M = naux, N = nd (groups of 8), inner = nao^2 cut into
// blocks of plen positions.
__device__ inline void project_tile(const double *__restrict__ B, const double *__restrict__ A,
                                    double *__restrict__ part, int naux, int nd, i64 npos, int plen,
                                    int tile, double *lds)
{
    typedef TileProject TL;
    const int nqt = cdiv_i(naux, kProjRows), nkg = cdiv_i(nd, 8);
    const int pb = tile / (nqt * nkg), rem = tile % (nqt * nkg);
    const int kg = rem / nqt, qt = rem % nqt;
    const i64 p0 = (i64)pb * plen;
    const int len = (int)((npos - p0) < plen ? (npos - p0) : plen);
    const int ndg = (nd - kg * 8) < 8 ? (nd - kg * 8) : 8;
    OpKC a{B + p0, npos, naux, len};
    OpKC b{A + (i64)kg * 8 * npos + p0, npos, ndg, len};
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, qt * kProjRows, 0, 0, len, lds, acc);
    const int ndp = nkg * 8;
    double *out = part + (i64)pb * naux * ndp;
    tile_foreach(acc, qt * kProjRows, 0, [&](int q, int kk, double v) {
        if (q < naux && kk < 8)
            out[(i64)q * ndp + kg * 8 + kk] = v;
    });
}

// The same product for 9 to 16 matrices A_k in one group (two sets of
// projections paired in one pass over B): part[pb][Q][k], k < 16, one tile per
// (position block, Q-tile).
__host__ __device__ inline int project16_tiles(int naux, int npb) { return cdiv_i(naux, kProjRows) * npb; }
__device__ inline void project16_tile(const double *__restrict__ B, const double *__restrict__ A,
                                      double *__restrict__ part, int naux, int nd, i64 npos,
                                      int plen, int tile, double *lds)
{
    typedef TileProject16 TL;
    const int nqt = cdiv_i(naux, kProjRows);
    const int pb = tile / nqt, qt = tile % nqt;
    const i64 p0 = (i64)pb * plen;
    const int len = (int)((npos - p0) < plen ? (npos - p0) : plen);
    OpKC a{B + p0, npos, naux, len};
    OpKC b{A + p0, npos, nd, len};
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, qt * kProjRows, 0, 0, len, lds, acc);
    double *out = part + (i64)pb * naux * 16;
    tile_foreach(acc, qt * kProjRows, 0, [&](int q, int kk, double v) {
        if (q < naux && kk < 16)
            out[(i64)q * 16 + kk] = v;
    });
}

// g[k][Q] = sum_{pb} part[pb][Q][k] in a fixed order.  A tile covers 64
// consecutive entries (Q, k) of one partial block; wave w of the four sums
// the blocks pb = w, w + 4, ... (coalesced 512-byte reads), and the four wave
// sums are added in wave order.
__device__ inline void reduce_tile(const double *__restrict__ part, double *__restrict__ g, int naux,
                                   int nd, int npb, int tile)
{
    __shared__ double red[4][64];
    const int ndp = cdiv_i(nd, 8) * 8;
    const i64 total = (i64)naux * ndp;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const i64 e = (i64)tile * 64 + lane;
    double s = 0.0;
    if (e < total) {
        const double *src = part + e;
        int pb = w;
        for (; pb + 12 < npb; pb += 16) {
            const double v0 = src[(i64)pb * total], v1 = src[(i64)(pb + 4) * total];
            const double v2 = src[(i64)(pb + 8) * total], v3 = src[(i64)(pb + 12) * total];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; pb < npb; pb += 4)
            s += src[(i64)pb * total];
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && e < total) {
        const int q = (int)(e / ndp), k = (int)(e % ndp);
        if (k < nd)
            g[(i64)k * naux + q] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    }
}

// ------------------------------------------------------------------ coulomb
// J[k][p] = sum_Q g[k][Q] B[Q][p] for the 8 densities of group kg and the 512
// positions of block pb: thread t takes positions pb*512 + t and + 256 (each
// load instruction reads 512 contiguous bytes), Q unrolled by 8, so 16 loads
// per thread are in flight.  The inner loop has no branches: positions past
// the end read a valid clamped address and densities past nd repeat the last
// one; neither is stored.  HBM-bound stream over B.
// J_k (+)= scale * sum_Q g[k][Q] B^Q (accumulate: add to what J holds).
__device__ inline void coulomb_tile(const double *__restrict__ B, const double *__restrict__ g,
                                    double *__restrict__ J, int naux, int nd, i64 npos, int tile,
                                    double scale = 1.0, int accumulate = 0)
{
    const int npb = cdiv_i(npos, 512);
    const int kg = tile / npb, pb = tile % npb;
    const int k0 = kg * 8;
    const int nk = (nd - k0) < 8 ? (nd - k0) : 8;
    const i64 p0 = (i64)pb * 512 + threadIdx.x, p1 = p0 + 256;
    const double *b0 = B + (p0 < npos ? p0 : npos - 1);
    const double *b1 = B + (p1 < npos ? p1 : npos - 1);
    const double *gk[8];
#pragma unroll
    for (int k = 0; k < 8; k++)
        gk[k] = g + (i64)(k0 + (k < nk ? k : nk - 1)) * naux;
    double a0[8], a1[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        a0[k] = 0.0;
        a1[k] = 0.0;
    }
    int q = 0;
    for (; q + 8 <= naux; q += 8) {
        double v0[8], v1[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            v0[u] = __builtin_nontemporal_load(b0 + (i64)(q + u) * npos);
            v1[u] = __builtin_nontemporal_load(b1 + (i64)(q + u) * npos);
        }
#pragma unroll
        for (int u = 0; u < 8; u++)
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const double gv = gk[k][q + u];
                a0[k] = fma(gv, v0[u], a0[k]);
                a1[k] = fma(gv, v1[u], a1[k]);
            }
    }
    for (; q < naux; q++) {
        const double v0 = b0[(i64)q * npos], v1 = b1[(i64)q * npos];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const double gv = gk[k][q];
            a0[k] = fma(gv, v0, a0[k]);
            a1[k] = fma(gv, v1, a1[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (k < nk) {
            double *Jk = J + (i64)(k0 + k) * npos;
            if (p0 < npos)
                Jk[p0] = accumulate ? Jk[p0] + scale * a0[k] : scale * a0[k];
            if (p1 < npos)
                Jk[p1] = accumulate ? Jk[p1] + scale * a1[k] : scale * a1[k];
        }
}

// ------------------------------------------------------------------ half-transform
// For slab Q = q0 + ql (ql < nq): XY[m][c] = sum_n B^Q[m][n] Cc[n][c], written
// as X_ws[k][m][ql*r + i] (c = k*r + i < R) or Y_ws[k][m][ql*r + i] (c - R),
// for the first ncol columns c (2R, or R when only X is needed).
// PACKED: B holds packed slabs (pk_size(nao) doubles each).
template <bool PACKED = false>
__device__ inline void ht_tile(const double *__restrict__ B, const double *__restrict__ Cc,
                               double *__restrict__ Xw, double *__restrict__ Yw, int nao, int nd,
                               int r, int q0, int ldw, int tile, double *lds, int ncol = -1)
{
    typedef TileHalf TL;
    const int R = nd * r, R2 = 2 * R;
    const int nc = ncol < 0 ? R2 : ncol;
    const int nmt = cdiv_i(nao, kHtM), nct = cdiv_i(nc, kHtN);
    const int ql = tile / (nmt * nct), rem = tile % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    const i64 n2 = PACKED ? pk_size(nao) : (i64)nao * nao;
    OpIC b{Cc, R2, nc, nao};
    Acc<TL> acc;
    acc.zero();
    if constexpr (PACKED) {
        OpPackedSym a{B + (i64)(q0 + ql) * n2, nao};
        tile_gemm<TL>(a, b, mb * kHtM, cb * kHtN, 0, nao, lds, acc);
    } else {
        OpKC a{B + (i64)(q0 + ql) * n2, nao, nao, nao};
        tile_gemm<TL>(a, b, mb * kHtM, cb * kHtN, 0, nao, lds, acc);
    }
    tile_foreach(acc, mb * kHtM, cb * kHtN, [&](int m, int c, double v) {
        if (m < nao && c < nc) {
            double *dst = c < R ? Xw : Yw;
            const int cc = c < R ? c : c - R;
            const int k = cc / r, i = cc % r;
            dst[((i64)k * nao + m) * ldw + (i64)ql * r + i] = v;
        }
    });
}

// The half-transform with an arbitrary tile shape TL of the 4x4x4 engine
// (full slabs).
template <class TL>
__device__ inline void ht_tile_tl(const double *__restrict__ B, const double *__restrict__ Cc,
                                  double *__restrict__ Xw, double *__restrict__ Yw, int nao, int nd,
                                  int r, int q0, int ldw, int tile, double *lds, int ncol)
{
    constexpr int BM = TL::BM, BN = TL::BN;
    const int R = nd * r, R2 = 2 * R;
    const int nc = ncol < 0 ? R2 : ncol;
    const int nmt = cdiv_i(nao, BM), nct = cdiv_i(nc, BN);
    const int ql = tile / (nmt * nct), rem = tile % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    const i64 n2 = (i64)nao * nao;
    OpKC a{B + (i64)(q0 + ql) * n2, nao, nao, nao};
    OpIC b{Cc, R2, nc, nao};
    auto out = [&](int m, int c, double v) {
        if (m < nao && c < nc) {
            double *dst = c < R ? Xw : Yw;
            const int cc = c < R ? c : c - R;
            const int k = cc / r, i = cc % r;
            dst[((i64)k * nao + m) * ldw + (i64)ql * r + i] = v;
        }
    };
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, mb * BM, cb * BN, 0, nao, lds, acc);
    tile_foreach(acc, mb * BM, cb * BN, out);
}

// The half-transform of the chunk's nq slabs as one product: the slabs,
// stacked, are an (nq nao) x nao matrix, so tile rows run across slab
// boundaries and no rows are padded per slab.  Row t of the stack is row
// t % nao of slab q0 + t / nao.  TL is a tile of the 16 x 16 x 4 engine; the
// chunk's slabs must span less than 4 GiB (buf_extent_ok).
template <class TL>
__host__ __device__ inline int ht_flat_tiles(int nao, int ncol, int nq)
{
    return cdiv_i((i64)nq * nao, TL::BM) * cdiv_i(ncol, TL::BN);
}
template <class TL>
__device__ inline void ht_tile_flat(const double *__restrict__ B, const double *__restrict__ Cc,
                                    double *__restrict__ Xw, double *__restrict__ Yw, int nao,
                                    int nd, int r, int q0, int nq, int ldw, int tile, double *lds,
                                    int ncol)
{
    constexpr int BM = TL::BM, BN = TL::BN;
    const int R = nd * r, R2 = 2 * R;
    const int nc = ncol < 0 ? R2 : ncol;
    const int rows = nq * nao;
    const int nct = cdiv_i(nc, BN);
    const int mb = tile / nct, cb = tile % nct;
    BufKC a{B + (i64)q0 * nao * nao, nao, rows, nao};
    BufIC b{Cc, R2, nc, nao};
    Acc16<TL> acc;
    acc.zero();
    // No inner-index masking: past row nao - 1, Cc reads zero (the end of its
    // resource), and the slab rows read there are finite data of the next row.
    tile_gemm16<TL, false>(a, b, mb * BM, cb * BN, 0, nao, lds, acc);
    // Output (t, c) goes to col(c)[row(t)]: col(c) = X_ws or Y_ws at density
    // k = c' / r, column i = c' % r (c' = c or c - R), and row(t) = m ldw +
    // ql r for t = ql nao + m.  A lane holds NB columns and 4 MA rows
    // (16 apart within 4 apart), decoded once each.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int rb = mb * BM + wr * TL::WM + (lane >> 4);
    const int cb0 = cb * BN + wc * TL::WN + (lane & 15);
    double *col[TL::NB];
    bool col_ok[TL::NB];
#pragma unroll
    for (int j = 0; j < TL::NB; j++) {
        const int c = cb0 + 16 * j;
        col_ok[j] = c < nc;
        const int cc = c < R ? c : c - R;
        const int k = cc / r, i = cc - k * r;
        col[j] = (c < R ? Xw : Yw) + (i64)k * nao * ldw + i;
    }
    const int ql0 = rb / nao, m0 = rb - ql0 * nao;
#pragma unroll
    for (int i = 0; i < TL::MA; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int d = 16 * i + 4 * v;
            if (rb + d < rows) {
                int m = m0 + d, ql = ql0;
                while (m >= nao) {
                    m -= nao;
                    ql++;
                }
                const i64 off = (i64)m * ldw + (i64)ql * r;
#pragma unroll
                for (int j = 0; j < TL::NB; j++)
                    if (col_ok[j])
                        col[j][off] = acc.c[i][j][v];
            }
        }
}

// The half-transform of packed slabs (jk.h JK_B_PACKED) on the 16 x 16 x 4
// engine: tiles per slab, the packed operand read in the form each stage
// allows (above, below or on the diagonal).  No inner-index mask: past row
// nao - 1, Cc reads zero and the packed reads are finite data or zero.
template <class TL>
__device__ inline void ht_tile16_packed(const double *__restrict__ B, const double *__restrict__ Cc,
                                        double *__restrict__ Xw, double *__restrict__ Yw, int nao,
                                        int nd, int r, int q0, int ldw, int tile, double *lds,
                                        int ncol)
{
    constexpr int BM = TL::BM, BN = TL::BN;
    const int R = nd * r, R2 = 2 * R;
    const int nc = ncol < 0 ? R2 : ncol;
    const int nmt = cdiv_i(nao, BM), nct = cdiv_i(nc, BN);
    const int ql = tile / (nmt * nct), rem = tile % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    BufPackedSym a{B + (i64)(q0 + ql) * pk_size(nao), nao};
    BufIC b{Cc, R2, nc, nao};
    Acc16<TL> acc;
    acc.zero();
    tile_gemm16<TL, false>(a, b, mb * BM, cb * BN, 0, nao, lds, acc);
    tile_foreach16(acc, mb * BM, cb * BN, [&](int m, int c, double v) {
        if (m < nao && c < nc) {
            double *dst = c < R ? Xw : Yw;
            const int cc = c < R ? c : c - R;
            const int k = cc / r, i = cc - k * r;
            dst[((i64)k * nao + m) * ldw + (i64)ql * r + i] = v;
        }
    });
}

// ------------------------------------------------------------------ exchange
// Kp[s][k][m][n] (+)= sum_{j in split s} X_ws[k][m][j] Y_ws[k][n][j]; the
// inner range [0, nj) is cut into nsplit contiguous pieces of jlen.
// With sym != 0 (Yw = Xw) only the tiles reaching n >= m are computed; the
// rest of K is filled by mirroring afterwards.
// Kp[split][k] (+)= scale * (the chunk's X Y^T over the split's inner range).
template <class TL = TileExch, bool MASK = true>
__device__ inline void ex_tile(const double *__restrict__ Xw, const double *__restrict__ Yw,
                               double *__restrict__ Kp, int nao, int nd, int nj, int ldw, int jlen,
                               int accumulate, int tile, double *lds, int sym = 0,
                               double scale = 1.0)
{
    static_assert(TL::BM == kExM && TL::BN == kExN, "exchange tile shape");
    const int nmt = cdiv_i(nao, kExM), nnt = cdiv_i(nao, kExN);
    const int pk = sym ? ex_tri_tiles(nao) : nmt * nnt;
    const int per = nd * pk;
    const int sp = tile / per;
    const int t = tile % per;
    const int k = t / pk, rem = t % pk;
    int mb, nb;
    if (sym) {
        ex_tri_coords(rem, nao, mb, nb);
    } else {
        mb = rem / nnt;
        nb = rem % nnt;
    }
    const int j0 = sp * jlen, j1 = (j0 + jlen) < nj ? (j0 + jlen) : nj;
    double *Kk = Kp + ((i64)sp * nd + k) * nao * nao;
    auto out = [&](int m, int n, double v) {
        if (m < nao && n < nao) {
            const i64 o = (i64)m * nao + n;
            Kk[o] = accumulate ? Kk[o] + scale * v : scale * v;
        }
    };
    if constexpr (TL::kMfma16) {
        // Resources end at column j1 of the last row.  MASK: inner indices
        // past j1 are zeroed in the last stage (needed unless every split
        // ends on a 16-deep stage boundary).
        BufKC a{Xw + (i64)k * nao * ldw, ldw, nao, j1};
        BufKC b{Yw + (i64)k * nao * ldw, ldw, nao, j1};
        Acc16<TL> acc;
        acc.zero();
        tile_gemm16<TL, MASK>(a, b, mb * kExM, nb * kExN, j0, j1, lds, acc);
        tile_update16(acc, mb * kExM, nb * kExN, Kk, nao, nao, nao, accumulate, scale);
    } else {
        OpKC a{Xw + (i64)k * nao * ldw, ldw, nao, j1};
        OpKC b{Yw + (i64)k * nao * ldw, ldw, nao, j1};
        Acc<TL> acc;
        acc.zero();
        tile_gemm<TL>(a, b, mb * kExM, nb * kExN, j0, j1, lds, acc);
        tile_foreach(acc, mb * kExM, nb * kExN, out);
    }
}

// out[e] = sum_{s < nsplit} part[s * n + e] (fixed order).
__device__ inline void sum_tile(const double *__restrict__ part, double *__restrict__ out, i64 n,
                                int nsplit, int tile)
{
    for (int u = 0; u < kElemTile / 256; u++) {
        const i64 e = (i64)tile * kElemTile + u * 256 + threadIdx.x;
        if (e < n) {
            double s = 0.0;
            for (int sp = 0; sp < nsplit; sp++)
                s += part[(i64)sp * n + e];
            out[e] = s;
        }
    }
}

} // namespace jk
