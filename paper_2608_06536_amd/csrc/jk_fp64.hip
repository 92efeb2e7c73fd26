// jk_fp64.hip -- FP64 kernels of the Cholesky-decomposed J/K build.
//
// The build (Sec. 2.3, Eq. (4), half-transform form K = B_V^T B_U):
//   pack          Cc[n][c]        = [C_L | C_R] re-laid as one nao x 2R matrix
//   density       D_k             = C_Lk C_Rk^T
//   project       part[p][Q][k]   = sum over a block of positions of B^Q . A_k
//   reduce        g[k][Q]         = sum of the partials in fixed order
//   coulomb       J_k             = sum_Q gamma_kQ B^Q
//   half-transform X^Q, Y^Q       = B^Q [C_L | C_R]            (per Q-chunk)
//   exchange      K_k            += sum_{Q in chunk} X^Q_k (Y^Q_k)^T
//
// Layouts of the chunk workspace: X_ws[k][m][ql*r + i] and Y_ws[k][n][ql*r + i]
// for the ql-th slab of the chunk, so that each row of the exchange operands
// is contiguous over the chunk's inner index (Q, i).
#include "f64_core.hpp"
#include "jk_kernels.hpp"

namespace jk {

// Tile shapes (chosen by measurement on MI355X): the half-transform uses
// 128 x 64 workgroup tiles of four 64 x 32 wave tiles (two workgroups per
// CU); the exchange product 128 x 64 tiles of eight 64 x 16 wave tiles (four
// waves per SIMD); the projection 256 Q-rows x 8 densities; the density
// 64 x 64.
constexpr int kHtM = 128, kHtN = 64;
constexpr int kExM = 128, kExN = 64;
constexpr int kProjRows = 256;
typedef Tile<kHtM, kHtN, 64, 32, 16> TileHalf;
typedef Tile<kExM, kExN, 64, 16, 16> TileExch;
typedef Tile<kProjRows, 8, 64, 8, 16> TileProject;
typedef Tile<64, 64, 32, 32, 16> TileDensity;

// ------------------------------------------------------------------ pack
__global__ void __launch_bounds__(256) k_pack_c(const double *__restrict__ CL,
                                                const double *__restrict__ CR, double *__restrict__ Cc,
                                                int nao, int nd, int r)
{
    const int R = nd * r, R2 = 2 * R;
    const i64 total = (i64)nao * R2;
    for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
        int n = (int)(e / R2), c = (int)(e % R2);
        const double *src = c < R ? CL : CR;
        int cc = c < R ? c : c - R;
        int k = cc / r, i = cc % r;
        Cc[e] = src[((i64)k * nao + n) * r + i];
    }
}

// ------------------------------------------------------------------ density
// D_k[m][n] = sum_i CL[k][m][i] CR[k][n][i]; grid: (tiles of nao x nao) x nd.
__global__ void __launch_bounds__(256) k_density(const double *__restrict__ CL,
                                                 const double *__restrict__ CR, double *__restrict__ D,
                                                 int nao, int r)
{
    typedef TileDensity TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    const int nt = (nao + 63) / 64;
    const int k = blockIdx.y;
    const int mb = blockIdx.x / nt, nb = blockIdx.x % nt;
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
// part[pb][Q][kk] = sum_{p in block pb} B[Q][p] * A[k0 + kk][p], kk < 8.
// A GEMM with M = naux, N = nd (in groups of 8), inner = nao^2 split into
// blocks of plen positions.  grid: x = Q tiles of kProjRows, y = density
// groups, z = position blocks.
__global__ void __launch_bounds__(256) k_project(const double *__restrict__ B,
                                                 const double *__restrict__ A, double *__restrict__ part,
                                                 int naux, int nd, i64 npos, int plen)
{
    typedef TileProject TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    const int qt = blockIdx.x, kg = blockIdx.y, pb = blockIdx.z;
    const i64 p0 = (i64)pb * plen;
    const int len = (int)((npos - p0) < plen ? (npos - p0) : plen);
    const int ndg = (nd - kg * 8) < 8 ? (nd - kg * 8) : 8;
    OpKC a{B + p0, npos, naux, len};
    OpKC b{A + (i64)kg * 8 * npos + p0, npos, ndg, len};
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, qt * kProjRows, 0, 0, len, lds, acc);
    const int ndp = ((nd + 7) / 8) * 8;
    double *out = part + (i64)pb * naux * ndp;
    tile_foreach(acc, qt * kProjRows, 0, [&](int q, int kk, double v) {
        if (q < naux && kk < 8)
            out[(i64)q * ndp + kg * 8 + kk] = v;
    });
}

// g[k][Q] = sum_{pb} part[pb][Q][k] (fixed order).
__global__ void __launch_bounds__(256) k_project_reduce(const double *__restrict__ part,
                                                        double *__restrict__ g, int naux, int nd,
                                                        int npb)
{
    const int ndp = ((nd + 7) / 8) * 8;
    const i64 total = (i64)naux * nd;
    for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
        int k = (int)(e / naux), q = (int)(e % naux);
        double s = 0.0;
        for (int pb = 0; pb < npb; pb++)
            s += part[((i64)pb * naux + q) * ndp + k];
        g[(i64)k * naux + q] = s;
    }
}

// ------------------------------------------------------------------ coulomb
// J[k][p] = sum_Q g[k][Q] B[Q][p] for k in [k0, k0 + 8); one position per
// thread, Q unrolled by 8 for loads in flight.  HBM-bound stream over B.
__global__ void __launch_bounds__(256) k_coulomb(const double *__restrict__ B,
                                                 const double *__restrict__ g, double *__restrict__ J,
                                                 int naux, int nd, int k0, i64 npos)
{
    const i64 p = (i64)blockIdx.x * 256 + threadIdx.x;
    const int nk = (nd - k0) < 8 ? (nd - k0) : 8;
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; k++)
        acc[k] = 0.0;
    const bool ok = p < npos;
    const double *bp = B + (ok ? p : 0);
    int q = 0;
    for (; q + 8 <= naux; q += 8) {
        double bv[8];
#pragma unroll
        for (int u = 0; u < 8; u++)
            bv[u] = ok ? __builtin_nontemporal_load(bp + (i64)(q + u) * npos) : 0.0;
#pragma unroll
        for (int u = 0; u < 8; u++)
#pragma unroll
            for (int k = 0; k < 8; k++)
                if (k < nk)
                    acc[k] = fma(g[(i64)(k0 + k) * naux + q + u], bv[u], acc[k]);
    }
    for (; q < naux; q++) {
        double b = ok ? bp[(i64)q * npos] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nk)
                acc[k] = fma(g[(i64)(k0 + k) * naux + q], b, acc[k]);
    }
    if (ok) {
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nk)
                J[(i64)(k0 + k) * npos + p] = acc[k];
    }
}

// ------------------------------------------------------------------ half-transform
// For slab Q = q0 + ql (ql < nq): XY[m][c] = sum_n B^Q[m][n] Cc[n][c], written
// as X_ws[k][m][ql*r + i] (c = k*r + i < R) or Y_ws[k][m][ql*r + i] (c - R).
// grid.x = nq * nmt * nct (XCD-swizzled), tile kHtM x kHtN.
__global__ void __launch_bounds__(256, 2) k_half_transform(const double *__restrict__ B,
                                                        const double *__restrict__ Cc,
                                                        double *__restrict__ Xw, double *__restrict__ Yw,
                                                        int nao, int nd, int r, int q0, int nq,
                                                        int ldw)
{
    typedef TileHalf TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    const int R = nd * r, R2 = 2 * R;
    const int nmt = (nao + kHtM - 1) / kHtM, nct = (R2 + kHtN - 1) / kHtN;
    const int ntile = nq * nmt * nct;
    const int t = xcd_swizzle(blockIdx.x, ntile);
    const int ql = t / (nmt * nct), rem = t % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    const i64 n2 = (i64)nao * nao;
    OpKC a{B + (i64)(q0 + ql) * n2, nao, nao, nao};
    OpIC b{Cc, R2, R2, nao};
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, mb * kHtM, cb * kHtN, 0, nao, lds, acc);
    tile_foreach(acc, mb * kHtM, cb * kHtN, [&](int m, int c, double v) {
        if (m < nao && c < R2) {
            double *dst = c < R ? Xw : Yw;
            int cc = c < R ? c : c - R;
            int k = cc / r, i = cc % r;
            dst[((i64)k * nao + m) * ldw + (i64)ql * r + i] = v;
        }
    });
}

// ------------------------------------------------------------------ exchange
// Kp[s][k][m][n] (+)= sum_{j in split s} X_ws[k][m][j] Y_ws[k][n][j], the inner
// range [0, nj) cut into nsplit contiguous pieces of jlen.  With nsplit == 1
// Kp is K itself.  grid.x = nsplit * nd * nmt * nnt (XCD-swizzled).
__global__ void __launch_bounds__(512, 4) k_exchange(const double *__restrict__ Xw,
                                                  const double *__restrict__ Yw, double *__restrict__ Kp,
                                                  int nao, int nd, int nj, int ldw, int nsplit,
                                                  int jlen, int accumulate)
{
    typedef TileExch TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    const int nmt = (nao + kExM - 1) / kExM, nnt = (nao + kExN - 1) / kExN;
    const int ntile = nsplit * nd * nmt * nnt;
    int t = xcd_swizzle(blockIdx.x, ntile);
    const int sp = t / (nd * nmt * nnt);
    t -= sp * (nd * nmt * nnt);
    const int k = t / (nmt * nnt), rem = t % (nmt * nnt);
    const int mb = rem / nnt, nb = rem % nnt;
    const int j0 = sp * jlen, j1 = (j0 + jlen) < nj ? (j0 + jlen) : nj;
    OpKC a{Xw + (i64)k * nao * ldw, ldw, nao, j1};
    OpKC b{Yw + (i64)k * nao * ldw, ldw, nao, j1};
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, mb * kExM, nb * kExN, j0, j1, lds, acc);
    double *Kk = Kp + ((i64)sp * nd + k) * nao * nao;
    tile_foreach(acc, mb * kExM, nb * kExN, [&](int m, int n, double v) {
        if (m < nao && n < nao) {
            i64 o = (i64)m * nao + n;
            Kk[o] = accumulate ? Kk[o] + v : v;
        }
    });
}

// out[e] = sum_{s < nsplit} part[s * n + e] (fixed order).
__global__ void __launch_bounds__(256) k_sum_splits(const double *__restrict__ part,
                                                    double *__restrict__ out, i64 n, int nsplit)
{
    for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < n; e += (i64)gridDim.x * 256) {
        double s = 0.0;
        for (int sp = 0; sp < nsplit; sp++)
            s += part[(i64)sp * n + e];
        out[e] = s;
    }
}

// ------------------------------------------------------------------ launchers

static inline int cdiv(i64 a, i64 b) { return (int)((a + b - 1) / b); }

int device_slots()
{
    static int slots = 0;
    if (slots == 0) {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            ncu <= 0)
            ncu = 256;
        slots = 2 * ncu;
    }
    return slots;
}

int pick_split(int tiles, int smax)
{
    const int slots = device_slots();
    if (smax < 1)
        smax = 1;
    int best = 1;
    double best_eff = -1.0;
    for (int s = 1; s <= smax; s++) {
        const i64 w = (i64)tiles * s;
        const i64 rounds = (w + slots - 1) / slots;
        const double eff = (double)w / (double)(rounds * slots);
        if (w >= slots && eff >= 0.9)
            return s;
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = s;
        }
    }
    return best;
}

hipError_t launch_pack_c(const double *CL, const double *CR, double *Cc, int nao, int nd, int r,
                         hipStream_t s)
{
    i64 total = (i64)nao * 2 * nd * r;
    int grid = cdiv(total, 256);
    if (grid > 65535)
        grid = 65535;
    {
        ProfScope ps_("pack_c", s);
        hipLaunchKernelGGL(k_pack_c, dim3(grid), dim3(256), 0, s, CL, CR, Cc, nao, nd, r);
    }
    return hipGetLastError();
}

hipError_t launch_density(const double *CL, const double *CR, double *D, int nao, int nd, int r,
                          hipStream_t s)
{
    int nt = cdiv(nao, 64);
    {
        ProfScope ps_("density", s);
        hipLaunchKernelGGL(k_density, dim3(nt * nt, nd), dim3(256), 0, s, CL, CR, D, nao, r);
    }
    return hipGetLastError();
}

int project_nblocks(i64 npos, int naux, int nd, int *plen)
{
    // Aim for >= 2048 workgroups in total; position blocks are multiples of 16.
    int nqt = cdiv(naux, kProjRows), nkg = cdiv(nd, 8);
    i64 want = 2048 / (nqt * nkg);
    if (want < 1)
        want = 1;
    i64 len = (npos + want - 1) / want;
    len = ((len + 15) / 16) * 16;
    if (len < 256)
        len = 256;
    *plen = (int)len;
    return cdiv(npos, len);
}

hipError_t launch_project(const double *B, const double *A, double *part, double *g, int naux,
                          int nd, i64 npos, hipStream_t s)
{
    int plen;
    int npb = project_nblocks(npos, naux, nd, &plen);
    dim3 grid(cdiv(naux, kProjRows), cdiv(nd, 8), npb);
    {
        ProfScope ps_("project", s);
        hipLaunchKernelGGL(k_project, grid, dim3(256), 0, s, B, A, part, naux, nd, npos, plen);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    i64 total = (i64)naux * nd;
    int rg = cdiv(total, 256);
    if (rg > 65535)
        rg = 65535;
    {
        ProfScope ps_("project_reduce", s);
        hipLaunchKernelGGL(k_project_reduce, dim3(rg), dim3(256), 0, s, part, g, naux, nd, npb);
    }
    return hipGetLastError();
}

hipError_t launch_coulomb(const double *B, const double *g, double *J, int naux, int nd, i64 npos,
                          hipStream_t s)
{
    for (int k0 = 0; k0 < nd; k0 += 8) {
        {
            ProfScope ps_("coulomb", s);
            hipLaunchKernelGGL(k_coulomb, dim3(cdiv(npos, 256)), dim3(256), 0, s, B, g, J, naux, nd, k0,
                           npos);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_half_transform(const double *B, const double *Cc, double *Xw, double *Yw,
                                 int nao, int nd, int r, int q0, int nq, int ldw, hipStream_t s)
{
    int nmt = cdiv(nao, kHtM), nct = cdiv(2 * (i64)nd * r, kHtN);
    {
        ProfScope ps_("half_transform", s);
        hipLaunchKernelGGL(k_half_transform, dim3(nq * nmt * nct), dim3(256), 0, s, B, Cc, Xw, Yw, nao,
                       nd, r, q0, nq, ldw);
    }
    return hipGetLastError();
}

int exchange_nsplit(int nao, int nd, int nj)
{
    // Full rounds of workgroups; each split keeps >= 256 inner indices.
    const int tiles = nd * cdiv(nao, kExM) * cdiv(nao, kExN);
    int maxs = nj / 256 > 1 ? nj / 256 : 1;
    if (maxs > 16)
        maxs = 16;
    return pick_split(tiles, maxs);
}

hipError_t launch_exchange(const double *Xw, const double *Yw, double *Kp, int nao, int nd, int nj,
                           int ldw, int nsplit, int accumulate, hipStream_t s)
{
    int jlen = cdiv(nj, nsplit);
    jlen = ((jlen + 15) / 16) * 16;
    {
        ProfScope ps_("exchange", s);
        hipLaunchKernelGGL(k_exchange, dim3(nsplit * nd * cdiv(nao, kExM) * cdiv(nao, kExN)),
                       dim3(TileExch::NTHR), 0, s, Xw, Yw, Kp, nao, nd,
                       nj, ldw, nsplit, jlen, accumulate);
    }
    return hipGetLastError();
}

hipError_t launch_sum_splits(const double *part, double *out, i64 n, int nsplit, hipStream_t s)
{
    int grid = cdiv(n, 256);
    if (grid > 65535)
        grid = 65535;
    {
        ProfScope ps_("sum_splits", s);
        hipLaunchKernelGGL(k_sum_splits, dim3(grid), dim3(256), 0, s, part, out, n, nsplit);
    }
    return hipGetLastError();
}

} // namespace jk
