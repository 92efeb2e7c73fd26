// coulomb_upper.hpp -- the HBM streams over B (gamma and J) from the upper
// triangles of the slabs.
//
// J_k = sum_Q gamma_kQ B^Q (Sec. 2.3, Eq. (4)) with every slab B^Q symmetric
// (a precondition of the engine): each J_k[m][n], m <= n, is a sum over the
// slabs of B^Q[m][n] only, and J_k[n][m] is the same sum.  Reading the upper
// triangle halves the bytes of this HBM-bound stream; each sum is written at
// both places.  Per position the slabs are taken in increasing Q, one fused
// multiply-add each, so a symmetric B gives the J of the full-square stream
// bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jk_tiles.hpp"

namespace jk {

// Row pair i of an nao x nao upper triangle: row i from its diagonal
// (nao - i positions), then row nao - 1 - i from its diagonal (i + 1
// positions): nao + 1 positions, so that all pairs weigh the same (the middle
// row of an odd nao stands alone).
__host__ __device__ inline int cu_pairs(int nao) { return (nao + 1) / 2; }
__host__ __device__ inline int cu_blocks(int nao) { return (nao + 1 + 255) / 256; }
__host__ __device__ inline int cu_tiles(int nao, int nd)
{
    return ((nd + 7) / 8) * cu_pairs(nao) * cu_blocks(nao);
}

// J_k (+)= scale * sum_Q g[k][Q] B^Q on the positions of one tile: 8 densities
// of group kg, 256 positions of one row pair (one per thread), slabs unrolled
// by 16 so that 16 loads per thread are in flight.
__device__ inline void coulomb_upper_tile(const double *__restrict__ B, const double *__restrict__ g,
                                          double *__restrict__ J, int nao, int naux, int nd,
                                          int tile, double scale = 1.0, int accumulate = 0)
{
    const int np = cu_pairs(nao), nb = cu_blocks(nao);
    const int kg = tile / (np * nb), rem = tile % (np * nb);
    const int i = rem / nb, blk = rem % nb;
    const int m1 = i, m2 = nao - 1 - i;
    const int len1 = nao - m1, len2 = m2 > m1 ? nao - m2 : 0;
    const int e = blk * 256 + (int)threadIdx.x;
    const bool live = e < len1 + len2;
    const int ee = live ? e : 0;                 // a valid address for the idle lanes
    const int m = ee < len1 ? m1 : m2;
    const int n = ee < len1 ? m1 + ee : m2 + (ee - len1);
    const int64_t npos = (int64_t)nao * nao;
    const double *b = B + (int64_t)m * nao + n;
    const int k0 = kg * 8;
    const int nk = (nd - k0) < 8 ? (nd - k0) : 8;
    const double *gk[8];
#pragma unroll
    for (int k = 0; k < 8; k++)
        gk[k] = g + (int64_t)(k0 + (k < nk ? k : nk - 1)) * naux;
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; k++)
        a[k] = 0.0;
    int q = 0;
    for (; q + 16 <= naux; q += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; u++)
            v[u] = __builtin_nontemporal_load(b + (int64_t)(q + u) * npos);
#pragma unroll
        for (int u = 0; u < 16; u++)
#pragma unroll
            for (int k = 0; k < 8; k++)
                a[k] = fma(gk[k][q + u], v[u], a[k]);
    }
    for (; q < naux; q++) {
        const double v = b[(int64_t)q * npos];
#pragma unroll
        for (int k = 0; k < 8; k++)
            a[k] = fma(gk[k][q], v, a[k]);
    }
    if (!live)
        return;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (k < nk) {
            double *Jk = J + (int64_t)(k0 + k) * npos;
            const int64_t p = (int64_t)m * nao + n, t = (int64_t)n * nao + m;
            Jk[p] = accumulate ? Jk[p] + scale * a[k] : scale * a[k];
            if (n != m)
                Jk[t] = accumulate ? Jk[t] + scale * a[k] : scale * a[k];
        }
}

// ------------------------------------------------------------------ gamma
// gamma_kQ = <B^Q, A_k> = sum_{m <= n} B^Q[m][n] S_k[m][n] with S_k the fold
// of A_k onto its upper triangle: A_k[m][n] + A_k[n][m] above the diagonal,
// A_k[m][m] on it, zero below (fold_upper_row, in place).  A product with
// M = naux, N = the matrices, inner = the upper-triangle positions: row m
// contributes columns m .. nao - 1.
//
// Rows go in groups of G consecutive rows m0 .. m0 + G - 1, each row one
// segment of the 4x4x4 engine's segmented pipeline starting at column m0 (a
// uniform stride of nao between segments) with depth nao - m0: the few
// positions left of a row's diagonal multiply the zeros of S, and every read
// stays in its row.  Groups are paired (g with ng - 1 - g) so that the tiles
// weigh the same; part[pair][Q][k] holds each pair's sums, added in a fixed
// order by reduce_tile.  About 512 workgroups in all: at nao 500 these tiles
// (groups of 4 rows) ran at 4.4 TB/s, groups of 1 and 2 rows (2000 and 1000
// tiles) at 4.1-4.2.
__host__ __device__ inline int pu_group_rows(int nao, int naux, int nkg)
{
    const int nqt = (naux + kProjRows - 1) / kProjRows;
    int want = 512 / (nqt * nkg);
    if (want < 1)
        want = 1;
    const int g = (nao + 2 * want - 1) / (2 * want);
    return g < 1 ? 1 : g;
}
__host__ __device__ inline int pu_pairs(int nao, int G) { return ((nao + G - 1) / G + 1) / 2; }

// In-place fold of row a of matrix k (nmat matrices of nao x nao): for
// b > a, A[a][b] += A[b][a] and A[b][a] = 0.  Each pair belongs to one row.
__device__ inline void fold_upper_row(double *__restrict__ A, int nao, int k, int a)
{
    double *Ak = A + (int64_t)k * nao * nao;
    for (int b = a + 1 + (int)threadIdx.x; b < nao; b += 256) {
        const double x = Ak[(int64_t)a * nao + b], y = Ak[(int64_t)b * nao + a];
        Ak[(int64_t)a * nao + b] = x + y;
        Ak[(int64_t)b * nao + a] = 0.0;
    }
}

// One tile: a pair of row groups, one Q-tile of kProjRows slabs, one group of
// 8 matrices (TL = TileProject, NK = 8: nd in groups of 8) or all of up to 16
// (TL = TileProject16, NK = 16: nd <= 16 in one group).
template <class TL, int NK>
__device__ inline void project_upper_tile(const double *__restrict__ B, const double *__restrict__ S,
                                          double *__restrict__ part, int naux, int nd, int nao,
                                          int G, int tile, double *lds)
{
    const int ng = (nao + G - 1) / G;
    const int nqt = cdiv_i(naux, kProjRows), nkg = NK == 8 ? cdiv_i(nd, 8) : 1;
    const int pb = tile / (nqt * nkg), rem = tile % (nqt * nkg);
    const int kg = rem / nqt, qt = rem % nqt;
    const int ndg = NK == 8 ? ((nd - kg * 8) < 8 ? (nd - kg * 8) : 8) : nd;
    const int64_t npos = (int64_t)nao * nao;
    Acc<TL> acc;
    acc.zero();
#pragma unroll 1
    for (int h = 0; h < 2; h++) {
        const int grp = h == 0 ? pb : ng - 1 - pb;
        if (h == 1 && grp <= pb)
            break;                                 // the middle group of an odd count
        const int m0 = grp * G;
        const int rows = (nao - m0) < G ? (nao - m0) : G;
        const int kdepth = nao - m0;
        OpKC a{B + (int64_t)m0 * nao + m0, npos, naux, kdepth};
        OpKC b{S + (int64_t)kg * 8 * npos + (int64_t)m0 * nao + m0, npos, ndg, kdepth};
        tile_gemm_seg<TL>(a, b, nao, nao, rows, qt * kProjRows, 0, kdepth, lds, acc);
    }
    const int ndp = NK == 8 ? nkg * 8 : 16;
    double *out = part + (int64_t)pb * naux * ndp;
    tile_foreach(acc, qt * kProjRows, 0, [&](int q, int kk, double v) {
        if (q < naux && kk < NK)
            out[(int64_t)q * ndp + kg * 8 + kk] = v;
    });
}

} // namespace jk
