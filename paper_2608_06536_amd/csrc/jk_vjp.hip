// jk_vjp.hip -- FP64 kernels of the reverse-mode derivative of the CD J/K
// build (Sec. 2.1, Eq. (1): the adjoint of J and K is J and K applied to the
// cotangent).  For L = sum_k <W_k, J_k> + <V_k, K_k> and symmetric B^Q:
//
//   omega_kQ = <W_k, B^Q>          (projection kernel, jk_fp64.hip)
//   X^Q_k = B^Q C_Lk, Y^Q_k = B^Q C_Rk     (recomputed per Q-chunk)
//   P^Q_k = V_k Y^Q_k,   R^Q_k = V_k^T X^Q_k                  (stage B)
//   dC_Lk = sum_Q B^Q (P^Q_k + omega_kQ C_Rk)                  (stage C)
//   dC_Rk = sum_Q B^Q (R^Q_k + omega_kQ C_Lk)
//   dB^Q  = sum_k gamma_kQ W_k + P^Q_k C_Lk^T + C_Rk (R^Q_k)^T
//                + omega_kQ C_Lk C_Rk^T                         (stage D)
//
// (omega_kQ Y^Q_k = B^Q omega_kQ C_Rk, so the omega terms of dC fold into the
// stage-C operand.)  Stage D is one product with inner dimension 3R:
//   [P^Q | C_R | omega C_L] [C_L | R^Q | C_R]^T
// plus the gamma W term added in its epilogue.
//
// Layouts: X/Y come from the half-transform kernel as X_ws[k][m][ql*r + i];
// stage B writes P/R per slab as Pq[ql][m][k*r + i] (ld R) so that stages C
// and D read all densities of a slab as one contiguous row.  Cc[n][c] is
// [C_L | C_R] with c < 2R; omx[Q][c] = omega_{c / r, Q} for c < R.
#include "f64_core.hpp"
#include "jk_kernels.hpp"

namespace jk {

namespace {
// 128 x 64 workgroup tiles of four 64 x 32 wave tiles (two workgroups per CU).
constexpr int kTM = 128, kTN = 64;
typedef Tile<kTM, kTN, 64, 32, 16> TileV;
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
// WHICH = 0: Pq[ql][m][k*r+i] = sum_n V_k[m][n] Y_ws[k][n][ql*r+i]
// WHICH = 1: Rq[ql][m][k*r+i] = sum_n V_k[n][m] X_ws[k][n][ql*r+i]
// grid.x = nd * nmt * njt (XCD-swizzled).
template <int WHICH>
__global__ void __launch_bounds__(256, 2) k_vjp_stage_b(const double *__restrict__ V,
                                                     const double *__restrict__ Zw,
                                                     double *__restrict__ Out, int nao, int nd, int r,
                                                     int nj, int ldw)
{
    typedef TileV TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    const int R = nd * r;
    const int nmt = (nao + kTM - 1) / kTM, njt = (nj + kTN - 1) / kTN;
    const int t = xcd_swizzle(blockIdx.x, nd * nmt * njt);
    const int k = t / (nmt * njt), rem = t % (nmt * njt);
    const int mb = rem / njt, jb = rem % njt;
    const double *Vk = V + (i64)k * nao * nao;
    OpIC b{Zw + (i64)k * nao * ldw, ldw, nj, nao};
    Acc<TL> acc;
    acc.zero();
    if (WHICH == 0) {
        OpKC a{Vk, nao, nao, nao};
        tile_gemm<TL>(a, b, mb * kTM, jb * kTN, 0, nao, lds, acc);
    } else {
        OpIC a{Vk, nao, nao, nao};
        tile_gemm<TL>(a, b, mb * kTM, jb * kTN, 0, nao, lds, acc);
    }
    tile_foreach(acc, mb * kTM, jb * kTN, [&](int m, int j, double v) {
        if (m < nao && j < nj) {
            int ql = j / r, i = j - ql * r;
            Out[((i64)ql * nao + m) * R + (i64)k * r + i] = v;
        }
    });
}

// ------------------------------------------------------------------ stage C
// Operand of stage C: element (c, n) for c < 2R of slab ql:
//   c <  R: Pq[ql][n][c]     + omx[Q][c]     * Cc[n][R + c]
//   c >= R: Rq[ql][n][c - R] + omx[Q][c - R] * Cc[n][c - R]
struct OpStageC {
    static constexpr bool kContig = false;
    static constexpr int NRAW = 3;
    const double *Pq, *Rq, *omx, *Cc;   // Pq/Rq already offset to slab ql, omx to row Q
    int nao, R;
    bool has_v, has_w;
    __device__ __forceinline__ void fetch(int c, int n, double *raw) const
    {
        const int R2 = 2 * R;
        const int cc0 = c < R2 ? c : R2 - 1;
        const int nn = n < nao ? n : nao - 1;
        const bool lo = cc0 < R;
        const int cc = lo ? cc0 : cc0 - R;
        raw[0] = has_v ? (lo ? Pq : Rq)[(i64)nn * R + cc] : 0.0;
        raw[1] = has_w ? omx[cc] : 0.0;
        raw[2] = has_w ? Cc[(i64)nn * R2 + (lo ? R + cc : cc)] : 0.0;
    }
    __device__ __forceinline__ double finish(int c, int n, const double *raw) const
    {
        if (c >= 2 * R || n >= nao)
            return 0.0;
        return fma(raw[1], raw[2], raw[0]);
    }
};

// dCp[sp][m][c] (+)= sum_{ql in split sp} sum_n B^{q0+ql}[m][n] op(c, n)
// grid.x = nsplit * nmt * nct.
__global__ void __launch_bounds__(256, 2) k_vjp_stage_c(const double *__restrict__ B,
                                                     const double *__restrict__ Pq,
                                                     const double *__restrict__ Rq,
                                                     const double *__restrict__ omx,
                                                     const double *__restrict__ Cc,
                                                     double *__restrict__ dCp, int nao, int R, int q0,
                                                     int nq, int nsplit, int qlen, int has_v,
                                                     int has_w, int accumulate)
{
    typedef TileV TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    const int R2 = 2 * R;
    const int nmt = (nao + kTM - 1) / kTM, nct = (R2 + kTN - 1) / kTN;
    const int t = xcd_swizzle(blockIdx.x, nsplit * nmt * nct);
    const int sp = t / (nmt * nct), rem = t % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    const i64 n2 = (i64)nao * nao;
    Acc<TL> acc;
    acc.zero();
    const int qa = sp * qlen, qb = (qa + qlen) < nq ? (qa + qlen) : nq;
    for (int ql = qa; ql < qb; ql++) {
        const int Q = q0 + ql;
        OpKC a{B + (i64)Q * n2, nao, nao, nao};
        OpStageC b{Pq + (i64)ql * nao * R, Rq + (i64)ql * nao * R, omx + (i64)Q * R, Cc, nao, R,
                   has_v != 0, has_w != 0};
        tile_gemm<TL>(a, b, mb * kTM, cb * kTN, 0, nao, lds, acc);
    }
    double *out = dCp + (i64)sp * nao * R2;
    tile_foreach(acc, mb * kTM, cb * kTN, [&](int m, int c, double v) {
        if (m < nao && c < R2) {
            i64 o = (i64)m * R2 + c;
            out[o] = accumulate ? out[o] + v : v;
        }
    });
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

// ------------------------------------------------------------------ stage D
// A(a, j): j < R: Pq[a][j];  j < 2R: Cc[a][j] (C_R);  j < 3R: omx[j-2R] Cc[a][j-2R] (omega C_L)
struct OpStageDA {
    static constexpr bool kContig = true;
    static constexpr int NRAW = 2;
    const double *Pq, *Cc, *omx;
    int nao, R, jhi;
    __device__ __forceinline__ void fetch(int a, int j, double *raw) const
    {
        const int aa = a < nao ? a : nao - 1;
        const int jj = j < jhi ? j : jhi - 1;
        const i64 row = (i64)aa * 2 * R;
        if (jj < R) {
            raw[0] = Pq[(i64)aa * R + jj];
            raw[1] = 1.0;
        } else if (jj < 2 * R) {
            raw[0] = Cc[row + jj];
            raw[1] = 1.0;
        } else {
            raw[0] = Cc[row + jj - 2 * R];
            raw[1] = omx[jj - 2 * R];
        }
    }
    __device__ __forceinline__ double finish(int a, int j, const double *raw) const
    {
        return (a < nao && j < jhi) ? raw[0] * raw[1] : 0.0;
    }
};
// B(b, j): j < R: Cc[b][j] (C_L);  j < 2R: Rq[b][j-R];  j < 3R: Cc[b][j-R] (C_R)
struct OpStageDB {
    static constexpr bool kContig = true;
    static constexpr int NRAW = 1;
    const double *Rq, *Cc;
    int nao, R, jhi;
    __device__ __forceinline__ void fetch(int b, int j, double *raw) const
    {
        const int bb = b < nao ? b : nao - 1;
        const int jj = j < jhi ? j : jhi - 1;
        const i64 row = (i64)bb * 2 * R;
        if (jj < R)
            raw[0] = Cc[row + jj];
        else if (jj < 2 * R)
            raw[0] = Rq[(i64)bb * R + jj - R];
        else
            raw[0] = Cc[row + jj - R];
    }
    __device__ __forceinline__ double finish(int b, int j, const double *raw) const
    {
        return (b < nao && j < jhi) ? raw[0] : 0.0;
    }
};

// dB[q0+ql][a][b] = sum_{j in [jlo, jhi)} A(a, j) B(b, j) + sum_k gamma[k][Q] W[k][a][b]
// grid.x = nq * nt * nt (XCD-swizzled).
__global__ void __launch_bounds__(256, 2) k_vjp_stage_d(const double *__restrict__ Pq,
                                                     const double *__restrict__ Rq,
                                                     const double *__restrict__ Cc,
                                                     const double *__restrict__ omx,
                                                     const double *__restrict__ gam,
                                                     const double *__restrict__ W,
                                                     double *__restrict__ dB, int nao, int nd, int r,
                                                     int naux, int q0, int nq, int jlo, int jhi,
                                                     int has_w)
{
    typedef TileV TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    const int R = nd * r;
    const int nmt = (nao + kTM - 1) / kTM, nnt = (nao + kTN - 1) / kTN;
    const int t = xcd_swizzle(blockIdx.x, nq * nmt * nnt);
    const int ql = t / (nmt * nnt), rem = t % (nmt * nnt);
    const int ab = rem / nnt, bb = rem % nnt;
    const int Q = q0 + ql;
    OpStageDA a{Pq + (i64)ql * nao * R, Cc, omx + (i64)Q * R, nao, R, jhi};
    OpStageDB b{Rq + (i64)ql * nao * R, Cc, nao, R, jhi};
    Acc<TL> acc;
    acc.zero();
    tile_gemm<TL>(a, b, ab * kTM, bb * kTN, jlo, jhi, lds, acc);
    const i64 n2 = (i64)nao * nao;
    double *out = dB + (i64)Q * n2;
    tile_foreach(acc, ab * kTM, bb * kTN, [&](int ia, int ib, double v) {
        if (ia < nao && ib < nao) {
            const i64 o = (i64)ia * nao + ib;
            if (has_w)
                for (int k = 0; k < nd; k++)
                    v = fma(gam[(i64)k * naux + Q], W[(i64)k * n2 + o], v);
            out[o] = v;
        }
    });
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

hipError_t launch_vjp_stage_b(const double *V, const double *Xw, const double *Yw, double *Pq,
                              double *Rq, int nao, int nd, int r, int nj, int ldw, hipStream_t s)
{
    const int nmt = cdiv(nao, kTM), njt = cdiv(nj, kTN);
    dim3 grid(nd * nmt * njt);
    {
        ProfScope ps_("vjp_stage_b_p", s);
        hipLaunchKernelGGL(k_vjp_stage_b<0>, grid, dim3(256), 0, s, V, Yw, Pq, nao, nd, r, nj, ldw);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("vjp_stage_b_r", s);
        hipLaunchKernelGGL(k_vjp_stage_b<1>, grid, dim3(256), 0, s, V, Xw, Rq, nao, nd, r, nj, ldw);
    }
    return hipGetLastError();
}

int vjp_stage_c_nsplit(int nao, int R, int qc)
{
    int tiles = cdiv(nao, kTM) * cdiv(2 * (i64)R, kTN);
    int ns = cdiv(512, tiles);
    if (ns > qc)
        ns = qc;
    return ns < 1 ? 1 : ns;
}

hipError_t launch_vjp_stage_c(const double *B, const double *Pq, const double *Rq,
                              const double *omx, const double *Cc, double *dCp, int nao, int R,
                              int q0, int nq, int nsplit, int has_v, int has_w, int accumulate,
                              hipStream_t s)
{
    const int nmt = cdiv(nao, kTM), nct = cdiv(2 * (i64)R, kTN);
    const int qlen = cdiv(nq, nsplit);
    {
        ProfScope ps_("vjp_stage_c", s);
        hipLaunchKernelGGL(k_vjp_stage_c, dim3(nsplit * nmt * nct), dim3(256), 0, s, B, Pq, Rq, omx, Cc,
                       dCp, nao, R, q0, nq, nsplit, qlen, has_v, has_w, accumulate);
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

hipError_t launch_vjp_stage_d(const double *Pq, const double *Rq, const double *Cc,
                              const double *omx, const double *gam, const double *W, double *dB,
                              int nao, int nd, int r, int naux, int q0, int nq, int has_v,
                              int has_w, hipStream_t s)
{
    const int R = nd * r;
    const int jlo = has_v ? 0 : 2 * R;
    const int jhi = has_w ? 3 * R : 2 * R;
    {
        ProfScope ps_("vjp_stage_d", s);
        hipLaunchKernelGGL(k_vjp_stage_d, dim3(nq * cdiv(nao, kTM) * cdiv(nao, kTN)), dim3(256), 0, s, Pq, Rq, Cc, omx, gam, W,
                       dB, nao, nd, r, naux, q0, nq, jlo, jhi > jlo ? jhi : jlo, has_w);
    }
    return hipGetLastError();
}

} // namespace jk
