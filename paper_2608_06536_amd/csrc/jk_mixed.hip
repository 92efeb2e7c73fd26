// jk_mixed.hip -- mixed-precision kernels of the CD J/K build.
//
// The bulk products (half-transforms and the exchange contraction) run as
// exact fixed-point slice products on the INT8 matrix cores (slice_core.hpp);
// gamma, J, every cross-chunk sum and the final K accumulation stay FP64.
//
//   slice   rows of an FP64 operand -> NS int8 digit planes + row exponent
//   ht      [X^Q | Y^Q] = slices(B^Q) x slices([C_L | C_R]), recombined in FP64
//   ex      K_k (+)= slices(X_k) x slices(Y_k) over the chunk, recombined in FP64
#include "jk_kernels.hpp"
#include "slice_core.hpp"

namespace jk {

namespace {
constexpr int kNS = 5;                  // digits per operand (35 bits)
constexpr int kMT = 64, kNT = 64;       // workgroup tile
typedef STile<kMT, kNT, kNS> TileS;

inline int cdiv(i64 a, i64 b) { return (int)((a + b - 1) / b); }
inline int grid_1d(i64 n)
{
    int g = cdiv(n, 256);
    return g > 65535 ? 65535 : (g < 1 ? 1 : g);
}
} // namespace

// ------------------------------------------------------------------ slicing
// Source element (b, m, k) = src[b * bs + m * rs + k * ks] for b < nb, m < nr,
// k < nk.  Output plane p, row b * rp + m, byte k at
// out[p * pstride + (b * rp + m) * kp + k]; rows m in [nr, rp) and bytes k in
// [nk, kp) are written as zero.  exps[b * rp + m] = row exponent.  One wave
// per output row.
__global__ void __launch_bounds__(256) k_slice_rows(const double *__restrict__ src, i64 bs, i64 rs,
                                                    i64 ks, int nb, int nr, int nk, int rp, int kp,
                                                    int8_t *__restrict__ out, i64 pstride,
                                                    int *__restrict__ exps)
{
    const int lane = threadIdx.x & 63;
    const i64 row = (i64)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (i64)nb * rp)
        return;
    const int b = (int)(row / rp), m = (int)(row % rp);
    int8_t *dst = out + row * kp;
    if (m >= nr) {
        for (int k = lane * 4; k < kp; k += 256) {
#pragma unroll
            for (int p = 0; p < kNS; p++)
                *(int *)(dst + p * pstride + k) = 0;
        }
        if (lane == 0)
            exps[row] = 0;
        return;
    }
    const double *s = src + (i64)b * bs + (i64)m * rs;
    double mx = 0.0;
    for (int k = lane; k < nk; k += 64)
        mx = fmax(mx, fabs(s[(i64)k * ks]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        mx = fmax(mx, __shfl_xor(mx, off));
    const int e = row_exponent(mx);
    if (lane == 0)
        exps[row] = e;
    // four consecutive bytes per lane and step
    for (int k0 = lane * 4; k0 < kp; k0 += 256) {
        int8_t d[4][kNS];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = k0 + u;
            const double v = k < nk ? s[(i64)k * ks] : 0.0;
            slice_value<kNS>(v, e, d[u]);
        }
#pragma unroll
        for (int p = 0; p < kNS; p++) {
            const int w = (d[0][p] & 0xff) | ((d[1][p] & 0xff) << 8) | ((d[2][p] & 0xff) << 16) |
                          ((int)(d[3][p] & 0xff) << 24);
            *(int *)(dst + p * pstride + k0) = w;
        }
    }
}

// ------------------------------------------------------------------ half-transform
// For slab ql of the chunk: XY[m][c] = 2^(eB + eC + 2) * sum_l S_l 2^(-7 l),
// written as X_ws[k][m][ql*r + i] (c = k*r + i < R) or Y_ws (c - R).
// A planes: rows ql * mp + m (ld kp); B planes: rows c (ld kp).
__global__ void __launch_bounds__(256) k_ht_mixed(const int8_t *__restrict__ Bp, i64 bpstride,
                                                  const int *__restrict__ eB,
                                                  const int8_t *__restrict__ Cp, i64 cpstride,
                                                  const int *__restrict__ eC, double *__restrict__ Xw,
                                                  double *__restrict__ Yw, int nao, int nd, int r,
                                                  int nq, int mp, int kp, int ldw)
{
    extern __shared__ char lds[];
    typedef TileS TL;
    const int R = nd * r, R2 = 2 * R;
    const int nmt = mp / kMT, nct = (R2 + kNT - 1) / kNT;
    const int t = blockIdx.x;
    const int ql = t / (nmt * nct), rem = t % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    SPlanes a{Bp + (i64)ql * mp * kp, bpstride, kp};
    SPlanes b{Cp, cpstride, kp};
    SAcc<TL> acc;
    acc.zero();
    stile_gemm<TL, kNS>(a, b, mb * kMT, cb * kNT, 0, kp, lds, acc);
#pragma unroll
    for (int e = 0; e < 16; e++) {
        int row, col;
        stile_coord<TL>(e, row, col);
        const int m = mb * kMT + row, c = cb * kNT + col;
        if (m < nao && c < R2) {
            const double v =
                ldexp(combine_levels<TL>(acc, e), eB[(i64)ql * mp + m] + eC[c] + 2);
            double *dst = c < R ? Xw : Yw;
            const int cc = c < R ? c : c - R;
            const int k = cc / r, i = cc % r;
            dst[((i64)k * nao + m) * ldw + (i64)ql * r + i] = v;
        }
    }
}

// ------------------------------------------------------------------ exchange
// Kp[s][k][m][n] (+)= 2^(eX + eY + 2) * sum_l S_l 2^(-7 l) over the inner
// range of split s.  X/Y planes: rows k * mp + m, ld jp.
__global__ void __launch_bounds__(256) k_ex_mixed(const int8_t *__restrict__ Xp,
                                                  const int8_t *__restrict__ Yp, i64 pstride,
                                                  const int *__restrict__ eX,
                                                  const int *__restrict__ eY, double *__restrict__ Kp,
                                                  int nao, int nd, int mp, int jp, int nsplit,
                                                  int jlen, int accumulate)
{
    extern __shared__ char lds[];
    typedef TileS TL;
    const int nt = mp / kMT;
    const int t = blockIdx.x;
    const int sp = t / (nd * nt * nt);
    const int rem0 = t % (nd * nt * nt);
    const int k = rem0 / (nt * nt), rem = rem0 % (nt * nt);
    const int mb = rem / nt, nb = rem % nt;
    const int j0 = sp * jlen, j1 = (j0 + jlen) < jp ? (j0 + jlen) : jp;
    SPlanes a{Xp + (i64)k * mp * jp, pstride, jp};
    SPlanes b{Yp + (i64)k * mp * jp, pstride, jp};
    SAcc<TL> acc;
    acc.zero();
    stile_gemm<TL, kNS>(a, b, mb * kMT, nb * kNT, j0, j1, lds, acc);
    double *Kk = Kp + ((i64)sp * nd + k) * nao * nao;
#pragma unroll
    for (int e = 0; e < 16; e++) {
        int row, col;
        stile_coord<TL>(e, row, col);
        const int m = mb * kMT + row, n = nb * kNT + col;
        if (m < nao && n < nao) {
            const double v =
                ldexp(combine_levels<TL>(acc, e), eX[(i64)k * mp + m] + eY[(i64)k * mp + n] + 2);
            const i64 o = (i64)m * nao + n;
            Kk[o] = accumulate ? Kk[o] + v : v;
        }
    }
}

// ------------------------------------------------------------------ launchers

int mixed_nslice() { return kNS; }
int mixed_row_pad() { return kMT; }
int mixed_k_pad() { return kSliceKP; }

hipError_t launch_slice_rows(const double *src, i64 bs, i64 rs, i64 ks, int nb, int nr, int nk,
                             int rp, int kp, int8_t *out, i64 pstride, int *exps, hipStream_t s)
{
    {
        ProfScope ps_("slice_rows", s);
        hipLaunchKernelGGL(k_slice_rows, dim3(cdiv((i64)nb * rp, 4)), dim3(256), 0, s, src, bs, rs, ks,
                           nb, nr, nk, rp, kp, out, pstride, exps);
    }
    return hipGetLastError();
}

// Dynamic LDS above 64 KB needs a per-kernel attribute; set once per process.
static hipError_t set_lds(const void *fn, bool &done)
{
    if (done)
        return hipSuccess;
    hipError_t e =
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, TileS::LDS_BYTES);
    if (e == hipSuccess)
        done = true;
    return e;
}
static bool g_lds_ht = false, g_lds_ex = false;

hipError_t launch_ht_mixed(const int8_t *Bp, i64 bpstride, const int *eB, const int8_t *Cp,
                           i64 cpstride, const int *eC, double *Xw, double *Yw, int nao, int nd,
                           int r, int nq, int mp, int kp, int ldw, hipStream_t s)
{
    hipError_t e = set_lds((const void *)k_ht_mixed, g_lds_ht);
    if (e != hipSuccess)
        return e;
    const int nmt = mp / kMT, nct = cdiv(2 * (i64)nd * r, kNT);
    {
        ProfScope ps_("ht_mixed", s);
        hipLaunchKernelGGL(k_ht_mixed, dim3(nq * nmt * nct), dim3(TileS::NTHR), TileS::LDS_BYTES, s, Bp,
                           bpstride, eB, Cp, cpstride, eC, Xw, Yw, nao, nd, r, nq, mp, kp, ldw);
    }
    return hipGetLastError();
}

int ex_mixed_nsplit(int mp, int nd, int jp)
{
    const int nt = mp / kMT;
    const int tiles = nd * nt * nt;
    int maxs = jp / 512 > 1 ? jp / 512 : 1;
    if (maxs > 16)
        maxs = 16;
    return pick_split(tiles, maxs);
}

hipError_t launch_ex_mixed(const int8_t *Xp, const int8_t *Yp, i64 pstride, const int *eX,
                           const int *eY, double *Kp, int nao, int nd, int mp, int jp, int nsplit,
                           int accumulate, hipStream_t s)
{
    hipError_t e = set_lds((const void *)k_ex_mixed, g_lds_ex);
    if (e != hipSuccess)
        return e;
    const int nt = mp / kMT;
    int jlen = cdiv(jp, nsplit);
    jlen = ((jlen + kSliceKP - 1) / kSliceKP) * kSliceKP;
    {
        ProfScope ps_("ex_mixed", s);
        hipLaunchKernelGGL(k_ex_mixed, dim3(nsplit * nd * nt * nt), dim3(TileS::NTHR), TileS::LDS_BYTES,
                           s, Xp, Yp, pstride, eX, eY, Kp, nao, nd, mp, jp, nsplit, jlen, accumulate);
    }
    return hipGetLastError();
}

} // namespace jk
