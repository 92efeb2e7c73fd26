// coulomb_upper.hpp -- the Coulomb matrix from the upper triangle of B.
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

} // namespace jk
