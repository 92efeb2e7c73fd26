// jk_vjp.hip -- FP64 kernels of the reverse-mode derivative of the CD J/K
// build (Sec. 2.1, Eq. (1): the adjoint of J and K is J and K applied to the
// cotangent).  For L = sum_k <W_k, J_k> + <V_k, K_k> and symmetric B^Q:
//
//   omega_kQ = <W_k, B^Q>, gamma_kQ = <D_k, B^Q>   (projection kernel)
//   X^Q_k = B^Q C_Lk, Y^Q_k = B^Q C_Rk              (recomputed per Q-chunk)
//   stage B:  P'^Q_k = V_k Y^Q_k   + omega_kQ C_Rk
//             R'^Q_k = V_k^T X^Q_k + omega_kQ C_Lk
//   stage C:  dC_Lk = sum_Q B^Q P'^Q_k,  dC_Rk = sum_Q B^Q R'^Q_k
//   stage D:  dB^Q  = sum_k C_Rk (R'^Q_k)^T + P'^Q_k C_Lk^T
//   affine:   dB^Q += sum_k gamma_kQ W_k + omega_kQ (D_k - 2 D_k^T)
//
// Stage C uses omega_kQ Y^Q_k = B^Q (omega_kQ C_Rk).  Stage D plus the affine
// term is the closed form sum_k gamma W + omega D + P C_L^T + C_R R^T
// rewritten with the primed factors: P' C_L^T + C_R R'^T = P C_L^T + C_R R^T
// + 2 omega D^T, hence E_k = D_k - 2 D_k^T.
//
// Layouts: X/Y come from the half-transform kernel as X_ws[k][m][ql*r + i].
// Each slab slot ql of the chunk owns one row-major block
//     L[ql][m][0:2R] = [ P' | R' ]      (column c = k*r + i per part)
// Stage C reads it whole; stage D is two products, C_R R'^T then P' C_L^T,
// with C_L and C_R read from Cc.  Cc[n][c] is [C_L | C_R] with c < 2R;
// omx[Q][c] = omega_{c / r, Q}, c < R.
#include "f64_core.hpp"
#include "f64_mfma16.hpp"
#include "jk_kernels.hpp"

namespace jk {

namespace {
// 128 x 64 workgroup tiles of four 64 x 32 wave tiles on the 16 x 16 x 4
// engine, three workgroups per CU (52 KB of dynamic LDS each).
constexpr int kTM = 128, kTN = 64;
typedef Tile16<kTM, kTN, 64, 32, 16> TileV;
} // namespace

// omx[Q][c] = om[c / r][Q], c < R.
__global__ void __launch_bounds__(256) k_omega_expand(const double *__restrict__ om,
                                                      double *__restrict__ omx, int naux, int nd,
                                                      int r)
{
    const int R = nd * r;
    const i64 total = (i64)naux * R;
    for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
        int q = (int)(e / R), c = (int)(e % R);
        omx[e] = om[(i64)(c / r) * naux + q];
    }
}

// ------------------------------------------------------------------ stage B
// WHICH = 0: L[ql][m][     k*r+i] = sum_n V_k[m][n] Y_ws[k][n][ql*r+i] + om * C_R
// WHICH = 1: L[ql][m][R  + k*r+i] = sum_n V_k[n][m] X_ws[k][n][ql*r+i] + om * C_L
// (om = omega_{k, q0+ql}; products skipped when has_v == 0, omega terms when
// has_w == 0).  grid.x = nd * nmt * njt (XCD-swizzled).
template <int WHICH>
__global__ void __launch_bounds__(256, 3) k_vjp_stage_b(const double *__restrict__ V,
                                                        const double *__restrict__ Zw,
                                                        const double *__restrict__ Cc,
                                                        const double *__restrict__ omx,
                                                        double *__restrict__ L, int nao, int nd,
                                                        int r, int q0, int nj, int ldw, int has_v,
                                                        int has_w)
{
    typedef TileV TL;
    extern __shared__ double lds[];
    const int R = nd * r, R2 = 2 * R;
    const int nmt = (nao + kTM - 1) / kTM, njt = (nj + kTN - 1) / kTN;
    const int t = xcd_swizzle(blockIdx.x, nd * nmt * njt);
    // row tiles fastest: the nmt tiles of a column block share its X/Y block,
    // read once from HBM while V_k's row panels stay in L2
    const int k = t / (nmt * njt), rem = t % (nmt * njt);
    const int jb = rem / nmt, mb = rem % nmt;
    Acc16<TL> acc;
    acc.zero();
    if (has_v) {
        const double *Vk = V + (i64)k * nao * nao;
        BufIC b{Zw + (i64)k * nao * ldw, ldw, nj, nao};
        if (WHICH == 0) {
            BufKC a{Vk, nao, nao, nao};
            tile_gemm16<TL>(a, b, mb * kTM, jb * kTN, 0, nao, lds, acc);
        } else {
            BufIC a{Vk, nao, nao, nao};
            tile_gemm16<TL>(a, b, mb * kTM, jb * kTN, 0, nao, lds, acc);
        }
    }
    // Output (m, j) goes to L at column block j: slot ql = j / r, column
    // c = k r + j % r, element ((ql nao + m) 2R + part + c); the omega term
    // adds omx[q0 + ql][c] * Cc[m][c or R + c].  A lane holds TL::NB columns
    // and 4 TL::MA rows, decoded once each.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / TL::WCOLS, wc = wave % TL::WCOLS;
    const int rb = mb * kTM + wr * TL::WM + (lane >> 4);
    const int cb0 = jb * kTN + wc * TL::WN + (lane & 15);
    i64 col_l[TL::NB];
    int col_cc[TL::NB];
    double col_om[TL::NB];
    bool col_ok[TL::NB];
#pragma unroll
    for (int jj = 0; jj < TL::NB; jj++) {
        const int j = cb0 + 16 * jj;
        col_ok[jj] = j < nj;
        const int ql = j / r, i = j - ql * r;
        const int c = k * r + i;
        col_l[jj] = (i64)ql * nao * R2 + (WHICH == 0 ? 0 : R) + c;
        col_cc[jj] = WHICH == 0 ? R + c : c;
        col_om[jj] = (has_w && col_ok[jj]) ? omx[(i64)(q0 + ql) * R + c] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < TL::MA; i++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int m = rb + 16 * i + 4 * v;
            if (m < nao) {
#pragma unroll
                for (int jj = 0; jj < TL::NB; jj++)
                    if (col_ok[jj]) {
                        double x = acc.c[i][jj][v];
                        if (has_w)
                            x = fma(col_om[jj], Cc[(i64)m * R2 + col_cc[jj]], x);
                        L[col_l[jj] + (i64)m * R2] = x;
                    }
            }
        }
}

// ------------------------------------------------------------------ stage C
// dCp[sp][m][c] (+)= sum_{ql in split sp} sum_n B^{q0+ql}[m][n] L[ql][n][c], c < 2R.
// grid.x = nsplit * nmt * nct.
__global__ void __launch_bounds__(256, 3) k_vjp_stage_c(const double *__restrict__ B,
                                                        const double *__restrict__ L,
                                                        double *__restrict__ dCp, int nao, int R,
                                                        int q0, int nq, int nsplit, int qlen,
                                                        int accumulate)
{
    typedef TileV TL;
    extern __shared__ double lds[];
    const int R2 = 2 * R;
    const int nmt = (nao + kTM - 1) / kTM, nct = (R2 + kTN - 1) / kTN;
    const int t = xcd_swizzle(blockIdx.x, nsplit * nmt * nct);
    const int sp = t / (nmt * nct), rem = t % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    const i64 n2 = (i64)nao * nao;
    Acc16<TL> acc;
    acc.zero();
    const int qa = sp * qlen, qb = (qa + qlen) < nq ? (qa + qlen) : nq;
    if (qb > qa) {
        // slabs qa..qb-1 as one pipelined sum, one resource per slab
        BufKC a{B + (i64)(q0 + qa) * n2, nao, nao, nao};
        BufIC b{L + (i64)qa * nao * R2, R2, R2, nao};
        tile_gemm16_seg<TL>(a, b, n2, (i64)nao * R2, qb - qa, mb * kTM, cb * kTN, nao, lds, acc);
    }
    tile_update16(acc, mb * kTM, cb * kTN, dCp + (i64)sp * nao * R2, R2, nao, R2, accumulate, 1.0);
}

// dCL[k][m][i] = sum_sp dCp[sp][m][k*r+i];  dCR[k][m][i] = sum_sp dCp[sp][m][R+k*r+i]
__global__ void __launch_bounds__(256) k_vjp_dc_finish(const double *__restrict__ dCp,
                                                       double *__restrict__ dCL,
                                                       double *__restrict__ dCR, int nao, int nd,
                                                       int r, int nsplit)
{
    const int R = nd * r, R2 = 2 * R;
    const i64 total = (i64)nao * R2;
    for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
        int m = (int)(e / R2), c = (int)(e % R2);
        double s = 0.0;
        for (int sp = 0; sp < nsplit; sp++)
            s += dCp[(i64)sp * total + e];
        double *dst = c < R ? dCL : dCR;
        int cc = c < R ? c : c - R;
        int k = cc / r, i = cc % r;
        dst[((i64)k * nao + m) * r + i] = s;
    }
}

// E[k][a][b] = D[k][a][b] - 2 D[k][b][a]
__global__ void __launch_bounds__(256) k_vjp_e_matrix(const double *__restrict__ D,
                                                      double *__restrict__ E, int nao, int nd)
{
    const i64 n2 = (i64)nao * nao, total = n2 * nd;
    for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
        const i64 k = e / n2, ab = e % n2;
        const int a = (int)(ab / nao), b = (int)(ab % nao);
        E[e] = D[e] - 2.0 * D[k * n2 + (i64)b * nao + a];
    }
}

// ------------------------------------------------------------------ stage D
// dB[q0+ql][a][b] = sum_{c<R} C_R[a][c] R'[ql][b][c] + sum_{c<R} P'[ql][a][c] C_L[b][c]
// (C_R[a][c] = Cc[a][R + c], C_L[b][c] = Cc[b][c]), the two sums in this order.
// grid.x = nq * nmt * nnt (XCD-swizzled).
__global__ void __launch_bounds__(256, 3) k_vjp_stage_d(const double *__restrict__ L,
                                                        const double *__restrict__ Cc,
                                                        double *__restrict__ dB, int nao, int R,
                                                        int q0, int nq)
{
    typedef TileV TL;
    extern __shared__ double lds[];
    const int R2 = 2 * R;
    const int nmt = (nao + kTM - 1) / kTM, nnt = (nao + kTN - 1) / kTN;
    const int t = xcd_swizzle(blockIdx.x, nq * nmt * nnt);
    const int ql = t / (nmt * nnt), rem = t % (nmt * nnt);
    const int ab = rem / nnt, bb = rem % nnt;
    const double *Lq = L + (i64)ql * nao * R2;
    Acc16<TL> acc;
    acc.zero();
    // The two products as two segments of one pipeline: segment g reads its
    // operands at the first segment's plus g times the distance between them
    // (both matrices have row length 2R, so their per-lane offsets agree).
    const double *a0 = Cc + R, *a1 = Lq, *b0 = Lq + R, *b1 = Cc;
    BufKC a{a0, R2, nao, R};
    BufKC b{b0, R2, nao, R};
    const i64 sa = ((i64)(intptr_t)a1 - (i64)(intptr_t)a0) / 8;
    const i64 sb = ((i64)(intptr_t)b1 - (i64)(intptr_t)b0) / 8;
    tile_gemm16_seg<TL>(a, b, sa, sb, 2, ab * kTM, bb * kTN, R, lds, acc);
    const i64 n2 = (i64)nao * nao;
    double *out = dB + (i64)(q0 + ql) * n2;
    tile_foreach16(acc, ab * kTM, bb * kTN, [&](int ia, int ib, double v) {
        if (ia < nao && ib < nao)
            out[(i64)ia * nao + ib] = v;
    });
}

// ------------------------------------------------------------------ packed B
// Packed-triangular slabs (jk.h JK_B_PACKED): element (a, b), a <= b, of slab
// Q at Q np + a nao - a (a - 1) / 2 + (b - a), np = nao (nao + 1) / 2.
__device__ __forceinline__ i64 pk_at(int a, int b, int nao)
{
    return (i64)a * (2 * (i64)nao - a + 1) / 2 + (b - a);
}

// Full squares of the chunk's packed slabs: out[ql][m][n] = B^{q0+ql}(min,
// max of m, n).  A workgroup takes one 32 x 32 tile pair (I <= J) of one
// slab through LDS, so that the tile and its mirror image are both written
// as coalesced rows.  grid.x = nq * ntri (ntri = nb (nb + 1) / 2 tile pairs).
constexpr int kUt = 32;
__global__ void __launch_bounds__(256) k_unpack_slabs(const double *__restrict__ Bp,
                                                      double *__restrict__ out, int nao, int q0,
                                                      int ntri)
{
    __shared__ double T[kUt][kUt + 1];
    const int nb = (nao + kUt - 1) / kUt;
    const int ql = blockIdx.x / ntri;
    int t = blockIdx.x % ntri, I = 0;
    while (t >= nb - I) {                      // row-major over the upper triangle
        t -= nb - I;
        I++;
    }
    const int J = I + t, m0 = I * kUt, n0 = J * kUt;
    const double *src = Bp + (i64)(q0 + ql) * ((i64)nao * (nao + 1) / 2);
    double *dst = out + (i64)ql * nao * nao;
    for (int e = threadIdx.x; e < kUt * kUt; e += 256) {
        const int i = e / kUt, j = e % kUt, m = m0 + i, n = n0 + j;
        if (m < nao && n < nao && m <= n)
            T[i][j] = src[pk_at(m, n, nao)];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kUt * kUt; e += 256) {
        const int i = e / kUt, j = e % kUt, m = m0 + i, n = n0 + j;
        if (m < nao && n < nao)
            dst[(i64)m * nao + n] = (I == J && j < i) ? T[j][i] : T[i][j];
    }
    if (I < J)
        for (int e = threadIdx.x; e < kUt * kUt; e += 256) {
            const int jj = e / kUt, ii = e % kUt, n = n0 + jj, m = m0 + ii;
            if (n < nao && m < nao)
                dst[(i64)n * nao + m] = T[ii][jj];
        }
}

// Upper-triangle tiles of the 128 x 64 grid: row tile ab covers column tiles
// 2 ab .. nnt - 1 (the first that meets columns >= its first row).
__device__ __forceinline__ int tri_first(int ab) { return ab * kTM / kTN; }
__host__ __device__ inline int vjp_tri_tiles(int nao)
{
    const int nmt = (nao + kTM - 1) / kTM, nnt = (nao + kTN - 1) / kTN;
    int n = 0;
    for (int ab = 0; ab < nmt; ab++)
        n += ab * kTM / kTN < nnt ? nnt - ab * kTM / kTN : 0;
    return n;
}

// Stage D for packed B.  The gradient with respect to the packed element
// (a, b), a < b, is dB[a][b] + dB[b][a], and dB[a][a] on the diagonal.  With
// A = [C_R | P'] and M = [R' | C_L] (dB = A M^T) the sum dB + dB^T =
// A M^T + M A^T is the product [A | M] [M | A]^T of depth 4R: the two
// products of the full stage D, then R' C_R^T + C_L P'^T, over the
// upper-triangle tiles only (the flops of the full dB), written to the packed
// positions; the diagonal is halved.  grid.x = nq * vjp_tri_tiles(nao).
__global__ void __launch_bounds__(256, 2) k_vjp_stage_d_packed(const double *__restrict__ L,
                                                               const double *__restrict__ Cc,
                                                               double *__restrict__ dB, int nao,
                                                               int R, int q0, int nq, int ntri)
{
    typedef TileV TL;
    extern __shared__ double lds[];
    const int R2 = 2 * R;
    const int t = xcd_swizzle(blockIdx.x, nq * ntri);
    const int ql = t / ntri;
    const int nnt = (nao + kTN - 1) / kTN;
    int tt = t % ntri, ab = 0;
    while (tt >= nnt - tri_first(ab)) {
        tt -= nnt - tri_first(ab);
        ab++;
    }
    const int bb = tri_first(ab) + tt;
    const double *Lq = L + (i64)ql * nao * R2;
    Acc16<TL> acc;
    acc.zero();
    {
        const double *a0 = Cc + R, *a1 = Lq, *b0 = Lq + R, *b1 = Cc;   // C_R R'^T + P' C_L^T
        BufKC a{a0, R2, nao, R};
        BufKC b{b0, R2, nao, R};
        tile_gemm16_seg<TL>(a, b, ((i64)(intptr_t)a1 - (i64)(intptr_t)a0) / 8,
                            ((i64)(intptr_t)b1 - (i64)(intptr_t)b0) / 8, 2, ab * kTM, bb * kTN, R,
                            lds, acc);
    }
    __syncthreads();                // the second pipeline refills the buffers the first read last
    {
        const double *a0 = Lq + R, *a1 = Cc, *b0 = Cc + R, *b1 = Lq;   // R' C_R^T + C_L P'^T
        BufKC a{a0, R2, nao, R};
        BufKC b{b0, R2, nao, R};
        tile_gemm16_seg<TL>(a, b, ((i64)(intptr_t)a1 - (i64)(intptr_t)a0) / 8,
                            ((i64)(intptr_t)b1 - (i64)(intptr_t)b0) / 8, 2, ab * kTM, bb * kTN, R,
                            lds, acc);
    }
    double *out = dB + (i64)(q0 + ql) * ((i64)nao * (nao + 1) / 2);
    tile_foreach16(acc, ab * kTM, bb * kTN, [&](int ia, int ib, double v) {
        if (ia <= ib && ib < nao)
            out[pk_at(ia, ib, nao)] = ia == ib ? 0.5 * v : v;
    });
}

// dB[Q][p] += sum_k gamma[k][Q] W[k][p] + omega[k][Q] E[k][p] for Q in
// [q0, q0 + nq): each thread keeps the W and E values of its two positions in
// registers across its slabs (densities in groups of 8) and updates four
// slabs at a time, so eight loads are in flight; blockIdx.y splits the
// chunk's slabs into ranges of qlen (each dB element has one owner).  No branches in
// the inner loop: a lone last position reuses a valid address and is not
// stored, densities past nd get zero weights.
__global__ void __launch_bounds__(256) k_vjp_db_affine(const double *__restrict__ gam,
                                                       const double *__restrict__ om,
                                                       const double *__restrict__ W,
                                                       const double *__restrict__ E,
                                                       double *__restrict__ dB, int nd, int naux,
                                                       i64 npos, int q0, int nq_all, int qlen)
{
    const i64 p0 = ((i64)blockIdx.x * 256 + threadIdx.x) * 2;
    const int qs = blockIdx.y * qlen;
    if (p0 >= npos || qs >= nq_all)
        return;
    q0 += qs;
    const int nq = (nq_all - qs) < qlen ? (nq_all - qs) : qlen;
    const bool two = p0 + 1 < npos;
    const i64 p1 = two ? p0 + 1 : p0;
    for (int k0 = 0; k0 < nd; k0 += 8) {
        const int nk = (nd - k0) < 8 ? (nd - k0) : 8;
        double w[8][2], e[8][2];
        const double *gk[8], *ok[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int kk = k0 + (k < nk ? k : 0);
            const i64 base = (i64)kk * npos;
            w[k][0] = W[base + p0];
            e[k][0] = E[base + p0];
            w[k][1] = W[base + p1];
            e[k][1] = E[base + p1];
            gk[k] = gam + (i64)kk * naux;
            ok[k] = om + (i64)kk * naux;
        }
        int ql = 0;
        for (; ql + 4 <= nq; ql += 4) {
            double v[4][2];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const double *d = dB + (i64)(q0 + ql + u) * npos;
                v[u][0] = d[p0];
                v[u][1] = d[p1];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int Q = q0 + ql + u;
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const double g = k < nk ? gk[k][Q] : 0.0, o = k < nk ? ok[k][Q] : 0.0;
                    v[u][0] = fma(g, w[k][0], fma(o, e[k][0], v[u][0]));
                    v[u][1] = fma(g, w[k][1], fma(o, e[k][1], v[u][1]));
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                double *d = dB + (i64)(q0 + ql + u) * npos;
                d[p0] = v[u][0];
                if (two)
                    d[p1] = v[u][1];
            }
        }
        for (; ql < nq; ql++) {
            const int Q = q0 + ql;
            double *d = dB + (i64)Q * npos;
            double v0 = d[p0], v1 = d[p1];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const double g = k < nk ? gk[k][Q] : 0.0, o = k < nk ? ok[k][Q] : 0.0;
                v0 = fma(g, w[k][0], fma(o, e[k][0], v0));
                v1 = fma(g, w[k][1], fma(o, e[k][1], v1));
            }
            d[p0] = v0;
            if (two)
                d[p1] = v1;
        }
    }
}

// ------------------------------------------------------------------ launchers

static inline int cdiv(i64 a, i64 b) { return (int)((a + b - 1) / b); }

static inline int grid_1d(i64 n)
{
    int g = cdiv(n, 256);
    return g > 65535 ? 65535 : (g < 1 ? 1 : g);
}

hipError_t launch_omega_expand(const double *om, double *omx, int naux, int nd, int r,
                               hipStream_t s)
{
    {
        ProfScope ps_("omega_expand", s);
        hipLaunchKernelGGL(k_omega_expand, dim3(grid_1d((i64)naux * nd * r)), dim3(256), 0, s, om, omx,
                       naux, nd, r);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_stage_b_one(int which, const double *V, const double *Zw, const double *Cc,
                                  const double *omx, double *L, int nao, int nd, int r, int q0,
                                  int nj, int ldw, int has_v, int has_w, hipStream_t s)
{
    const int nmt = cdiv(nao, kTM), njt = cdiv(nj, kTN);
    dim3 grid(nd * nmt * njt);
    const int lds = (int)sizeof(double) * TileV::LDS_DOUBLES;
    const void *fn = which ? (const void *)k_vjp_stage_b<1> : (const void *)k_vjp_stage_b<0>;
    hipError_t e = set_dynamic_lds(fn, lds);
    if (e != hipSuccess)
        return e;
    if (which) {
        ProfScope ps_("vjp_stage_b_r", s);
        hipLaunchKernelGGL(k_vjp_stage_b<1>, grid, dim3(TileV::NTHR), lds, s, V, Zw, Cc, omx, L, nao, nd,
                           r, q0, nj, ldw, has_v, has_w);
    } else {
        ProfScope ps_("vjp_stage_b_p", s);
        hipLaunchKernelGGL(k_vjp_stage_b<0>, grid, dim3(TileV::NTHR), lds, s, V, Zw, Cc, omx, L, nao, nd,
                           r, q0, nj, ldw, has_v, has_w);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_stage_b(const double *V, const double *Xw, const double *Yw,
                              const double *Cc, const double *omx, double *L, int nao, int nd,
                              int r, int q0, int nj, int ldw, int has_v, int has_w, hipStream_t s)
{
    const int nmt = cdiv(nao, kTM), njt = cdiv(nj, kTN);
    dim3 grid(nd * nmt * njt);
    const int lds = (int)sizeof(double) * TileV::LDS_DOUBLES;
    hipError_t e = set_dynamic_lds((const void *)k_vjp_stage_b<0>, lds);
    if (e == hipSuccess)
        e = set_dynamic_lds((const void *)k_vjp_stage_b<1>, lds);
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("vjp_stage_b_p", s);
        hipLaunchKernelGGL(k_vjp_stage_b<0>, grid, dim3(TileV::NTHR), lds, s, V, Yw, Cc, omx, L, nao, nd,
                           r, q0, nj, ldw, has_v, has_w);
    }
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("vjp_stage_b_r", s);
        hipLaunchKernelGGL(k_vjp_stage_b<1>, grid, dim3(TileV::NTHR), lds, s, V, Xw, Cc, omx, L, nao, nd,
                           r, q0, nj, ldw, has_v, has_w);
    }
    return hipGetLastError();
}

int vjp_stage_c_nsplit(int nao, int R, int qc)
{
    const int tiles = cdiv(nao, kTM) * cdiv(2 * (i64)R, kTN);
    // three workgroups per CU
    return pick_split_slots(tiles, qc < 64 ? qc : 64, device_slots() / 2 * 3);
}

hipError_t launch_vjp_stage_c(const double *B, const double *L, double *dCp, int nao, int R,
                              int q0, int nq, int nsplit, int accumulate, hipStream_t s)
{
    const int nmt = cdiv(nao, kTM), nct = cdiv(2 * (i64)R, kTN);
    const int qlen = cdiv(nq, nsplit);
    const int lds = (int)sizeof(double) * TileV::LDS_DOUBLES;
    hipError_t e = set_dynamic_lds((const void *)k_vjp_stage_c, lds);
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("vjp_stage_c", s);
        hipLaunchKernelGGL(k_vjp_stage_c, dim3(nsplit * nmt * nct), dim3(TileV::NTHR), lds, s, B, L, dCp,
                           nao, R, q0, nq, nsplit, qlen, accumulate);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_dc_finish(const double *dCp, double *dCL, double *dCR, int nao, int nd,
                                int r, int nsplit, hipStream_t s)
{
    {
        ProfScope ps_("vjp_dc_finish", s);
        hipLaunchKernelGGL(k_vjp_dc_finish, dim3(grid_1d((i64)nao * 2 * nd * r)), dim3(256), 0, s, dCp,
                           dCL, dCR, nao, nd, r, nsplit);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_e_matrix(const double *D, double *E, int nao, int nd, hipStream_t s)
{
    {
        ProfScope ps_("vjp_e_matrix", s);
        hipLaunchKernelGGL(k_vjp_e_matrix, dim3(grid_1d((i64)nao * nao * nd)), dim3(256), 0, s, D, E,
                           nao, nd);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_stage_d(const double *L, const double *Cc, double *dB, int nao, int R,
                              int q0, int nq, hipStream_t s)
{
    const int lds = (int)sizeof(double) * TileV::LDS_DOUBLES;
    hipError_t e = set_dynamic_lds((const void *)k_vjp_stage_d, lds);
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("vjp_stage_d", s);
        const dim3 g(nq * cdiv(nao, kTM) * cdiv(nao, kTN));
        hipLaunchKernelGGL(k_vjp_stage_d, g, dim3(TileV::NTHR), lds, s, L, Cc, dB, nao, R, q0, nq);
    }
    return hipGetLastError();
}

hipError_t launch_unpack_slabs(const double *Bp, double *out, int nao, int q0, int nq,
                               hipStream_t s)
{
    const int nb = cdiv(nao, kUt), ntri = nb * (nb + 1) / 2;
    {
        ProfScope ps_("vjp_unpack_slabs", s);
        hipLaunchKernelGGL(k_unpack_slabs, dim3(nq * ntri), dim3(256), 0, s, Bp, out, nao, q0, ntri);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_stage_d_packed(const double *L, const double *Cc, double *dB, int nao, int R,
                                     int q0, int nq, hipStream_t s)
{
    const int lds = (int)sizeof(double) * TileV::LDS_DOUBLES;
    hipError_t e = set_dynamic_lds((const void *)k_vjp_stage_d_packed, lds);
    if (e != hipSuccess)
        return e;
    const int ntri = vjp_tri_tiles(nao);
    {
        ProfScope ps_("vjp_stage_d", s);
        hipLaunchKernelGGL(k_vjp_stage_d_packed, dim3(nq * ntri), dim3(TileV::NTHR), lds, s, L, Cc, dB,
                           nao, R, q0, nq, ntri);
    }
    return hipGetLastError();
}

hipError_t launch_vjp_db_affine(const double *gam, const double *om, const double *W,
                                const double *E, double *dB, int nd, int naux, i64 npos, int q0,
                                int nq, hipStream_t s)
{
    {
        ProfScope ps_("vjp_db_affine", s);
        // enough workgroups to keep several in flight per CU
        const int nx = cdiv((npos + 1) / 2, 256);
        int ny = cdiv(4096, nx);
        if (ny > nq)
            ny = nq;
        if (ny < 1)
            ny = 1;
        const int qlen = cdiv(nq, ny);
        hipLaunchKernelGGL(k_vjp_db_affine, dim3(nx, cdiv(nq, qlen)), dim3(256), 0, s, gam, om, W, E,
                           dB, nd, naux, npos, q0, nq, qlen);
    }
    return hipGetLastError();
}

} // namespace jk
