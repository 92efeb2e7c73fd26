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
constexpr int kMT = 128, kNT = 64;      // workgroup tile (eight 32 x 32 waves)
constexpr int kKBS = 2;                 // 32-byte inner blocks per pipeline stage
constexpr int kRowPad = 128;            // plane rows are padded to this
constexpr int kKPad = kKBS * kSliceKB;  // plane inner bytes are padded to this
constexpr unsigned kExpBias = 2048;     // biased exponent code: 0 = no nonzero value
typedef STile<kMT, kNT, kNS, kKBS> TileS;

inline int cdiv(i64 a, i64 b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ int decode_exp(unsigned u) { return u ? (int)u - (int)kExpBias : 0; }

// Biased code of the exponent e with |v| < 2^e, 2^(e-1) <= |v| (0 for v = 0).
__device__ __forceinline__ unsigned exp_code(double v)
{
    int e;
    frexp(v, &e);
    return v != 0.0 ? (unsigned)(e + (int)kExpBias) : 0u;
}

__device__ __forceinline__ void write_digits(int8_t *dst, i64 pstride, const int8_t (*d)[kNS])
{
#pragma unroll
    for (int p = 0; p < kNS; p++) {
        const int w = (d[0][p] & 0xff) | ((d[1][p] & 0xff) << 8) | ((d[2][p] & 0xff) << 16) |
                      ((int)(d[3][p] & 0xff) << 24);
        *(int *)(dst + p * pstride) = w;
    }
}
} // namespace

// ------------------------------------------------------------------ slicing
// All slicers read source element (b, m, k) = src[b * bs + m * rs + k * ks]
// for b < nb, m < nr, k < nk and write the digit planes of rows b * rp + m in
// the K-blocked layout of slice_core.hpp; rows m in [nr, rp) and inner bytes
// k in [nk, 32 nkb) get zero digits.

// Generic two-pass slicer (any strides; used for the small [C_L | C_R]
// operand): 8 threads per row, 32 rows per workgroup, exps[b * rp + m] = row
// exponent.
__global__ void __launch_bounds__(256) k_slice_rows(const double *__restrict__ src, i64 bs, i64 rs,
                                                    i64 ks, int nb, int nr, int nk, int rp, int nkb,
                                                    int8_t *__restrict__ out, i64 pstride,
                                                    i64 kbstride, int *__restrict__ exps)
{
    const int t = threadIdx.x, sub = t & 7;
    const i64 row = (i64)blockIdx.x * 32 + (t >> 3);
    if (row >= (i64)nb * rp)        // whole 8-lane row groups leave together
        return;
    const int b = (int)(row / rp), m = (int)(row % rp);
    const bool live = m < nr;
    const double *s = src + (i64)b * bs + (i64)m * rs;
    double mx = 0.0;
    if (live)
        for (int k = sub; k < nk; k += 8)
            mx = fmax(mx, fabs(s[(i64)k * ks]));
    mx = fmax(mx, __shfl_xor(mx, 1));
    mx = fmax(mx, __shfl_xor(mx, 2));
    mx = fmax(mx, __shfl_xor(mx, 4));
    const int e = row_exponent(mx);
    if (sub == 0)
        exps[row] = live ? e : 0;
    int8_t *dst = out + row * kSliceKB + sub * 4;
    for (int kb = 0; kb < nkb; kb++) {
        int8_t d[4][kNS];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = kb * kSliceKB + sub * 4 + u;
            const double v = (live && k < nk) ? s[(i64)k * ks] : 0.0;
            slice_value<kNS>(v, e, d[u]);
        }
        write_digits(dst + (i64)kb * kbstride, pstride, d);
    }
}

// One-pass slicer for unit-stride rows of at most 256 * NJ elements: one wave
// per row holds the row in registers (lane l: elements 4 l + 256 j + u),
// reduces the maximum across the wave, then writes the digits.  Also clears
// clr[0 .. nclr) (the exponent codes that the following half-transform
// accumulates).
template <int NJ>
__global__ void __launch_bounds__(256) k_slice_rows_wave(const double *__restrict__ src, i64 bs,
                                                         i64 rs, int nb, int nr, int nk, int rp,
                                                         int nkb, int8_t *__restrict__ out,
                                                         i64 pstride, i64 kbstride,
                                                         int *__restrict__ exps,
                                                         unsigned *__restrict__ clr, int nclr)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < nclr; i += gridDim.x * 256)
        clr[i] = 0u;
    const int lane = threadIdx.x & 63;
    const i64 row = (i64)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (i64)nb * rp)        // whole waves leave together
        return;
    const int b = (int)(row / rp), m = (int)(row % rp);
    const bool live = m < nr;
    const double *s = src + (i64)b * bs + (i64)m * rs;
    double v[NJ][4];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < NJ; j++)
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = 256 * j + 4 * lane + u;
            v[j][u] = (live && k < nk) ? s[k] : 0.0;
            mx = fmax(mx, fabs(v[j][u]));
        }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        mx = fmax(mx, __shfl_xor(mx, o));
    const int e = row_exponent(mx);
    if (lane == 0)
        exps[row] = live ? e : 0;
    int8_t *dst = out + row * kSliceKB + 4 * (lane & 7);
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int kb = 8 * j + (lane >> 3);
        if (kb < nkb) {
            int8_t d[4][kNS];
#pragma unroll
            for (int u = 0; u < 4; u++)
                slice_value<kNS>(v[j][u], e, d[u]);
            write_digits(dst + (i64)kb * kbstride, pstride, d);
        }
    }
}

// Elementwise slicer for rows whose exponents are already known (biased
// codes ux[b * rp + m], see exp_code): unit-stride rows, 32 rows x one
// 32-byte inner block per workgroup (grid: row groups x nkb); each plane
// write of a workgroup is one contiguous kilobyte.
__global__ void __launch_bounds__(256) k_slice_elem(const double *__restrict__ src, i64 bs, i64 rs,
                                                    int nb, int nr, int nk, int rp,
                                                    int8_t *__restrict__ out, i64 pstride,
                                                    i64 kbstride, const unsigned *__restrict__ ux)
{
    const int t = threadIdx.x, sub = t & 7;
    const i64 row = (i64)blockIdx.x * 32 + (t >> 3);
    const int kb = blockIdx.y;
    if (row >= (i64)nb * rp)
        return;
    const int b = (int)(row / rp), m = (int)(row % rp);
    const bool live = m < nr;
    const int e = live ? decode_exp(ux[row]) : 0;
    const double *s = src + (i64)b * bs + (i64)m * rs;
    int8_t d[4][kNS];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int k = kb * kSliceKB + sub * 4 + u;
        const double v = (live && k < nk) ? s[k] : 0.0;
        slice_value<kNS>(v, e, d[u]);
    }
    write_digits(out + (i64)kb * kbstride + row * kSliceKB + sub * 4, pstride, d);
}

// ------------------------------------------------------------------ half-transform
// For slab ql of the chunk: XY[m][c] = 2^(eB + eC + 2) * sum_l S_l 2^(-7 l),
// written as X_ws[k][m][ql*r + i] (c = k*r + i < R) or Y_ws (c - R).
// A planes: rows ql * mp + m; B planes: rows c.  The epilogue also raises
// ux[key * mp + m] (key = c / r: X_k for key < nd, Y_(key-nd) above) to the
// exponent code of every value it writes: after all slabs of the chunk, ux
// holds the row exponents the X/Y slicer needs.  Columns of one key are
// contiguous, so a segmented max-scan over the 32 lanes of a row precedes
// one atomic per (row, key) segment.
__global__ void __launch_bounds__(512) k_ht_mixed(const int8_t *__restrict__ Bp, i64 bpstride,
                                                  i64 bkbstride, const int *__restrict__ eB,
                                                  const int8_t *__restrict__ Cp, i64 cpstride,
                                                  i64 ckbstride, const int *__restrict__ eC,
                                                  double *__restrict__ Xw, double *__restrict__ Yw,
                                                  unsigned *__restrict__ ux, int nao, int nd, int r,
                                                  int mp, int cp, int nkb, int ldw)
{
    extern __shared__ char lds[];
    typedef TileS TL;
    const int R = nd * r, R2 = 2 * R;
    const int nmt = mp / kMT, nct = cp / kNT;
    const int t = blockIdx.x;
    const int ql = t / (nmt * nct), rem = t % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    SPlanes a{Bp + (i64)ql * mp * kSliceKB, bpstride, bkbstride};
    SPlanes b{Cp, cpstride, ckbstride};
    SAcc<TL> acc;
    acc.zero();
    stile_gemm<TL, kNS>(a, b, mb * kMT, cb * kNT, 0, nkb, lds, acc);

    const int lane = threadIdx.x & 63, l32 = lane & 31;
    int row0, col;
    stile_coord<TL>(0, row0, col);
    const int c = cb * kNT + col;
    const int key = c < R2 ? c / r : -1;
    // segment structure of the 32 columns held by this half-wave
    int kup[5];
#pragma unroll
    for (int s = 0; s < 5; s++)
        kup[s] = __shfl_up(key, 1 << s, 32);
    const int knext = __shfl_down(key, 1, 32);
    const bool seg_end = l32 == 31 || knext != key;
#pragma unroll
    for (int e = 0; e < 16; e++) {
        int row, cl;
        stile_coord<TL>(e, row, cl);
        const int m = mb * kMT + row;
        const bool ok = m < nao && key >= 0;
        double v = 0.0;
        if (ok) {
            v = ldexp(combine_levels<TL>(acc, e), eB[(i64)ql * mp + m] + eC[c] + 2);
            double *dst = c < R ? Xw : Yw;
            const int cc = c < R ? c : c - R;
            const int k = cc / r, i = cc % r;
            dst[((i64)k * nao + m) * ldw + (i64)ql * r + i] = v;
        }
        unsigned code = ok ? exp_code(v) : 0u;
#pragma unroll
        for (int s = 0; s < 5; s++) {
            const unsigned o = __shfl_up(code, 1 << s, 32);
            if (l32 >= (1 << s) && kup[s] == key)
                code = o > code ? o : code;
        }
        if (ok && seg_end && code != 0u)
            atomicMax(ux + (i64)key * mp + m, code);
    }
}

// ------------------------------------------------------------------ exchange
// Kp[s][k][m][n] (+)= 2^(eX + eY + 2) * sum_l S_l 2^(-7 l) over the inner
// blocks [s * kbl, (s + 1) * kbl) of split s.  X/Y planes: rows k * mp + m;
// exponent codes ux[k * mp + m] (X) and uy[k * mp + n] (Y).
__global__ void __launch_bounds__(512) k_ex_mixed(const int8_t *__restrict__ Xp,
                                                  const int8_t *__restrict__ Yp, i64 pstride,
                                                  i64 kbstride, const unsigned *__restrict__ ux,
                                                  const unsigned *__restrict__ uy,
                                                  double *__restrict__ Kp, int nao, int nd, int mp,
                                                  int nkb, int kbl, int accumulate)
{
    extern __shared__ char lds[];
    typedef TileS TL;
    const int nmt = mp / kMT, nnt = mp / kNT;
    const int per = nd * nmt * nnt;
    const int t = blockIdx.x;
    const int sp = t / per, rem0 = t % per;
    const int k = rem0 / (nmt * nnt), rem = rem0 % (nmt * nnt);
    const int mb = rem / nnt, nb = rem % nnt;
    const int kb0 = sp * kbl < nkb ? sp * kbl : nkb;
    const int kb1 = (kb0 + kbl) < nkb ? (kb0 + kbl) : nkb;
    SPlanes a{Xp + (i64)k * mp * kSliceKB, pstride, kbstride};
    SPlanes b{Yp + (i64)k * mp * kSliceKB, pstride, kbstride};
    SAcc<TL> acc;
    acc.zero();
    stile_gemm<TL, kNS>(a, b, mb * kMT, nb * kNT, kb0, kb1, lds, acc);
    double *Kk = Kp + ((i64)sp * nd + k) * nao * nao;
#pragma unroll
    for (int e = 0; e < 16; e++) {
        int row, col;
        stile_coord<TL>(e, row, col);
        const int m = mb * kMT + row, n = nb * kNT + col;
        if (m < nao && n < nao) {
            const double v = ldexp(combine_levels<TL>(acc, e),
                                   decode_exp(ux[(i64)k * mp + m]) + decode_exp(uy[(i64)k * mp + n]) + 2);
            const i64 o = (i64)m * nao + n;
            Kk[o] = accumulate ? Kk[o] + v : v;
        }
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(unsigned *__restrict__ p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        p[i] = 0u;
}

// ------------------------------------------------------------------ launchers
int mixed_nslice() { return kNS; }
int mixed_row_pad() { return kRowPad; }
int mixed_k_pad() { return kKPad; }
int mixed_k_block() { return kSliceKB; }

hipError_t launch_slice_rows(const double *src, i64 bs, i64 rs, i64 ks, int nb, int nr, int nk,
                             int rp, int nkb, int8_t *out, i64 pstride, i64 kbstride, int *exps,
                             hipStream_t s)
{
    {
        ProfScope ps_("slice_rows", s);
        hipLaunchKernelGGL(k_slice_rows, dim3(cdiv((i64)nb * rp, 32)), dim3(256), 0, s, src, bs, rs,
                           ks, nb, nr, nk, rp, nkb, out, pstride, kbstride, exps);
    }
    return hipGetLastError();
}

hipError_t launch_slice_b(const double *src, i64 bs, i64 rs, int nb, int nr, int nk, int rp, int nkb,
                          int8_t *out, i64 pstride, i64 kbstride, int *exps, unsigned *clr, int nclr,
                          hipStream_t s)
{
    const int nj = cdiv(nkb, 8);
    const dim3 g(cdiv((i64)nb * rp, 4));
    {
        ProfScope ps_("slice_b", s);
        if (nj <= 1)
            hipLaunchKernelGGL(k_slice_rows_wave<1>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps, clr, nclr);
        else if (nj <= 2)
            hipLaunchKernelGGL(k_slice_rows_wave<2>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps, clr, nclr);
        else if (nj <= 4)
            hipLaunchKernelGGL(k_slice_rows_wave<4>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps, clr, nclr);
        else if (nj <= 8)
            hipLaunchKernelGGL(k_slice_rows_wave<8>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps, clr, nclr);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nj <= 8)
        return e;
    // long rows: generic two-pass slicer plus a separate clear
    e = launch_slice_rows(src, bs, rs, 1, nb, nr, nk, rp, nkb, out, pstride, kbstride, exps, s);
    if (e != hipSuccess || nclr <= 0)
        return e;
    hipLaunchKernelGGL(k_fill_u32, dim3(cdiv(nclr, 256)), dim3(256), 0, s, clr, nclr);
    return hipGetLastError();
}

hipError_t launch_slice_elem(const double *src, i64 bs, i64 rs, int nb, int nr, int nk, int rp,
                             int nkb, int8_t *out, i64 pstride, i64 kbstride, const unsigned *ux,
                             hipStream_t s)
{
    {
        ProfScope ps_("slice_xy", s);
        hipLaunchKernelGGL(k_slice_elem, dim3(cdiv((i64)nb * rp, 32), nkb), dim3(256), 0, s, src, bs,
                           rs, nb, nr, nk, rp, out, pstride, kbstride, ux);
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

hipError_t launch_ht_mixed(const int8_t *Bp, i64 bpstride, i64 bkbstride, const int *eB,
                           const int8_t *Cp, i64 cpstride, i64 ckbstride, const int *eC, double *Xw,
                           double *Yw, unsigned *ux, int nao, int nd, int r, int nq, int mp, int cp,
                           int nkb, int ldw, hipStream_t s)
{
    hipError_t e = set_lds((const void *)k_ht_mixed, g_lds_ht);
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("ht_mixed", s);
        hipLaunchKernelGGL(k_ht_mixed, dim3(nq * (mp / kMT) * (cp / kNT)), dim3(TileS::NTHR),
                           TileS::LDS_BYTES, s, Bp, bpstride, bkbstride, eB, Cp, cpstride, ckbstride,
                           eC, Xw, Yw, ux, nao, nd, r, mp, cp, nkb, ldw);
    }
    return hipGetLastError();
}

int ex_mixed_nsplit(int mp, int nd, int nkb)
{
    const int tiles = nd * (mp / kMT) * (mp / kNT);
    int maxs = nkb / 16 > 1 ? nkb / 16 : 1;
    if (maxs > 16)
        maxs = 16;
    return pick_split(tiles, maxs);
}

hipError_t launch_ex_mixed(const int8_t *Xp, const int8_t *Yp, i64 pstride, i64 kbstride,
                           const unsigned *ux, const unsigned *uy, double *Kp, int nao, int nd, int mp,
                           int nkb, int nsplit, int accumulate, hipStream_t s)
{
    hipError_t e = set_lds((const void *)k_ex_mixed, g_lds_ex);
    if (e != hipSuccess)
        return e;
    int kbl = cdiv(nkb, nsplit);
    kbl = cdiv(kbl, kKBS) * kKBS;
    {
        ProfScope ps_("ex_mixed", s);
        hipLaunchKernelGGL(k_ex_mixed, dim3(nsplit * nd * (mp / kMT) * (mp / kNT)), dim3(TileS::NTHR),
                           TileS::LDS_BYTES, s, Xp, Yp, pstride, kbstride, ux, uy, Kp, nao, nd, mp, nkb,
                           kbl, accumulate);
    }
    return hipGetLastError();
}

} // namespace jk
