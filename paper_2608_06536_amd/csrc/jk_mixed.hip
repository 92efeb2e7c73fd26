// jk_mixed.hip -- mixed-precision kernels of the CD J/K build.
//
// The bulk products (half-transforms and the exchange contraction) run as
// exact fixed-point slice products on the INT8 matrix cores (slice_core.hpp);
// gamma, J, every cross-chunk sum and the final K accumulation stay FP64.
//
//   slice   rows of an FP64 operand -> NS int8 digit planes + row exponent
//   ht      [X^Q | Y^Q] = slices(B^Q) x slices([C_L | C_R]), recombined in FP64
//   rowmax  exponent of every row (side, k, m) of X/Y over the chunk
//   ex      K_k (+)= slices(X_k) x slices(Y_k) over the chunk, recombined in FP64
#include <mutex>
#include <set>
#include <utility>

#include "jk_batched.hpp"
#include "jk_kernels.hpp"
#include "jk_tiles.hpp"
#include "slice_core.hpp"

namespace jk {

namespace {
constexpr int kNS = kSliceDigits;       // digits per operand (31 bits)
constexpr int kMT = 128, kNT = 128;     // workgroup tile: eight waves of 32 x 64
constexpr int kWTN = 2;                 // MFMA tiles per wave, side by side
constexpr int kRowPad = 128;            // plane rows are padded to this
constexpr int kKPad = kSliceKB;         // plane inner bytes are padded to this
typedef STileW<kMT, kNT, kNS, kWTN> TileS;   // exchange: eight waves, one workgroup per CU
constexpr int kHtMT = 64;                     // half-transform: 64 x 128, four waves,
typedef STileW<kHtMT, kNT, kNS, kWTN> TileH;  // two workgroups per CU
constexpr int kNbHt = 3, kNbEx = 3;           // LDS stage buffers
typedef SPipe<TileH, kNbHt> PipeHt;
typedef SPipe<TileS, kNbEx> PipeEx;

inline int cdiv(i64 a, i64 b) { return (int)((a + b - 1) / b); }

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
// operand): 8 threads per row (sub = lane & 7), exps[row] = row exponent.
__device__ __forceinline__ void slice_row8(const double *__restrict__ src, i64 bs, i64 rs, i64 ks,
                                           int nr, int nk, int rp, int nkb,
                                           int8_t *__restrict__ out, i64 pstride, i64 kbstride,
                                           int *__restrict__ exps, i64 row, int sub)
{
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
            slice_value(v, e, d[u]);
        }
        write_digits(dst + (i64)kb * kbstride, pstride, d);
    }
}

// 32 rows per workgroup.
__global__ void __launch_bounds__(256) k_slice_rows(const double *__restrict__ src, i64 bs, i64 rs,
                                                    i64 ks, int nb, int nr, int nk, int rp, int nkb,
                                                    int8_t *__restrict__ out, i64 pstride,
                                                    i64 kbstride, int *__restrict__ exps)
{
    const int t = threadIdx.x;
    const i64 row = (i64)blockIdx.x * 32 + (t >> 3);
    if (row >= (i64)nb * rp)        // whole 8-lane row groups leave together
        return;
    slice_row8(src, bs, rs, ks, nr, nk, rp, nkb, out, pstride, kbstride, exps, row, t & 7);
}

// One-pass slicer for unit-stride rows of at most 256 * NJ elements: one wave
// per row holds the row in registers (lane l: elements 4 l + 256 j + u),
// reduces the maximum across the wave, then writes the digits.
template <int NJ>
__device__ __forceinline__ void slice_row_wave(const double *__restrict__ src, i64 bs, i64 rs,
                                               int nr, int nk, int rp, int nkb,
                                               int8_t *__restrict__ out, i64 pstride, i64 kbstride,
                                               int *__restrict__ exps, i64 row)
{
    const int lane = threadIdx.x & 63;
    const int b = (int)(row / rp), m = (int)(row % rp);
    const bool live = m < nr;
    // loads are unconditional (clamped addresses), masked afterwards; rows
    // that start on 16 bytes with nk % 4 == 0 use 16-byte loads
    const double *s = src + (i64)b * bs + (i64)(live ? m : nr - 1) * rs;
    const bool vec = ((((uintptr_t)s) & 15) == 0) && (nk & 3) == 0;
    double v[NJ][4];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int k0 = 256 * j + 4 * lane;
        double x[4];
        if (vec) {
            const int kc = k0 < nk ? k0 : nk - 4;
            const double2 lo = *(const double2 *)(s + kc), hi = *(const double2 *)(s + kc + 2);
            x[0] = lo.x;
            x[1] = lo.y;
            x[2] = hi.x;
            x[3] = hi.y;
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++)
                x[u] = s[(k0 + u) < nk ? k0 + u : nk - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            v[j][u] = (live && k0 + u < nk) ? x[u] : 0.0;
            mx = fmax(mx, fabs(v[j][u]));
        }
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
                slice_value(v[j][u], e, d[u]);
            write_digits(dst + (i64)kb * kbstride, pstride, d);
        }
    }
}

template <int NJ>
__global__ void __launch_bounds__(256) k_slice_rows_wave(const double *__restrict__ src, i64 bs,
                                                         i64 rs, int nb, int nr, int nk, int rp,
                                                         int nkb, int8_t *__restrict__ out,
                                                         i64 pstride, i64 kbstride,
                                                         int *__restrict__ exps)
{
    const i64 row = (i64)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= (i64)nb * rp)        // whole waves leave together
        return;
    slice_row_wave<NJ>(src, bs, rs, nr, nk, rp, nkb, out, pstride, kbstride, exps, row);
}

// The same for packed symmetric slabs (jk.h JK_B_PACKED).  A workgroup takes
// a band of kBand rows [m0, m0 + kBand) of one slab and first gathers it into
// LDS with coalesced reads: the part n >= m of row m is contiguous in packed
// row m; the part n < m is column m of packed row n, and the band's kBand
// columns of packed row n are contiguous.  Wave w then slices rows w, w + 4
// of the band from LDS exactly as the one-pass slicer does.  nk = nr = nao.
constexpr int kBand = 8;

// Band [m0, m0 + kBand) of packed slab P, plane rows b * rp + m; T holds
// kBand x nao doubles of LDS.
template <int NJ>
__device__ __forceinline__ void slice_band_packed(const double *__restrict__ P, int b, int m0,
                                                  int nao, int rp, int nkb,
                                                  int8_t *__restrict__ out, i64 pstride,
                                                  i64 kbstride, int *__restrict__ exps, double *T)
{
    const int ld = nao;
    const int tid = threadIdx.x;
#pragma unroll 1
    for (int r = 0; r < kBand; r++) {          // n >= m: packed row m
        const int m = m0 + r;
        if (m < nao) {
            const double *row = P + pk_row(m, nao) - m;
            for (int n = m + tid; n < nao; n += 256)
                T[r * ld + n] = row[n];
        }
    }
    const int nlow = (m0 + kBand < nao ? m0 + kBand : nao) * kBand;
    for (int t = tid; t < nlow; t += 256) {    // n < m: column m of packed row n
        const int n = t / kBand, r = t % kBand, m = m0 + r;
        if (n < m && m < nao)
            T[r * ld + n] = P[pk_row(n, nao) + (m - n)];
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll 1
    for (int r = wave; r < kBand; r += 4) {
        const int m = m0 + r;
        if (m >= rp)
            break;
        const bool live = m < nao;
        const i64 row = (i64)b * rp + m;
        double v[NJ][4];
        double mx = 0.0;
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int k0 = 256 * j + 4 * lane;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int k = k0 + u;
                v[j][u] = (live && k < nao) ? T[r * ld + k] : 0.0;
                mx = fmax(mx, fabs(v[j][u]));
            }
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
                    slice_value(v[j][u], e, d[u]);
                write_digits(dst + (i64)kb * kbstride, pstride, d);
            }
        }
    }
}

template <int NJ>
__global__ void __launch_bounds__(256) k_slice_band_packed(const double *__restrict__ src, i64 bs,
                                                           int nb, int nao, int rp, int nkb,
                                                           int8_t *__restrict__ out, i64 pstride,
                                                           i64 kbstride, int *__restrict__ exps)
{
    extern __shared__ double T[];              // [kBand][nao]
    const int nband = (rp + kBand - 1) / kBand;
    const int b = blockIdx.x / nband, m0 = (blockIdx.x % nband) * kBand;
    slice_band_packed<NJ>(src + (i64)b * bs, b, m0, nao, rp, nkb, out, pstride, kbstride, exps, T);
}

// Elementwise slicer of the half-transformed factors.  Source XY[ql][m][c]
// (c < nkey r; X_k = columns k*r.., Y_k = columns R + k*r..; nkey = 2 nd, or
// nd when only X is formed), plane row (side * nd + k) * mp + m, inner index j = ql * r + i (j < nj), row
// exponents exps[plane row] known.  32 plane rows x one 32-byte inner block
// per workgroup (grid: row groups x nkb); each plane write of a workgroup is
// one contiguous kilobyte.
__device__ __forceinline__ void slice_xy_block(const double *__restrict__ XY, int nao, int nkey,
                                               int r, int mp, int nj, int8_t *__restrict__ out,
                                               i64 pstride, i64 kbstride,
                                               const int *__restrict__ exps, int row, int sub,
                                               int kb)
{
    const int key = row / mp, m = row % mp;
    const bool live = m < nao;
    const int e = exps[row];
    const i64 R2 = (i64)nkey * r;     // row length of XY
    // loads are unconditional (clamped addresses), masked afterwards
    const double *s = XY + (i64)(live ? m : nao - 1) * R2 + (i64)key * r;
    const int j0 = kb * kSliceKB + sub * 4;
    double x[4];
    const int q0 = j0 / r, i0 = j0 - q0 * r;
    const double *p0 = s + (i64)q0 * nao * R2 + i0;
    if (j0 + 3 < nj && i0 + 3 < r && (((uintptr_t)p0) & 15) == 0) {
        const double2 lo = *(const double2 *)p0, hi = *(const double2 *)(p0 + 2);
        x[0] = lo.x;
        x[1] = lo.y;
        x[2] = hi.x;
        x[3] = hi.y;
    } else {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int j = (j0 + u) < nj ? (j0 + u) : nj - 1;
            const int ql = j / r, i = j - ql * r;
            x[u] = s[(i64)ql * nao * R2 + i];
        }
    }
    int8_t d[4][kNS];
#pragma unroll
    for (int u = 0; u < 4; u++)
        slice_value((live && j0 + u < nj) ? x[u] : 0.0, e, d[u]);
    write_digits(out + (i64)kb * kbstride + (i64)row * kSliceKB + sub * 4, pstride, d);
}

__global__ void __launch_bounds__(256) k_slice_xy(const double *__restrict__ XY, int nao, int nkey,
                                                  int r, int mp, int nj, int8_t *__restrict__ out,
                                                  i64 pstride, i64 kbstride,
                                                  const int *__restrict__ exps, int nkb)
{
    const int t = threadIdx.x, sub = t & 7;
    const int row = blockIdx.x * 32 + (t >> 3);
    if (row >= nkey * mp)
        return;
    // inner blocks kb = blockIdx.y, + gridDim.y, ... (grid y is capped at 65535)
    for (int kb = blockIdx.y; kb < nkb; kb += gridDim.y)
        slice_xy_block(XY, nao, nkey, r, mp, nj, out, pstride, kbstride, exps, row, sub, kb);
}

// ------------------------------------------------------------------ half-transform
// For slab ql of the chunk: XY[ql][m][c] = 2^(eB + eC - 14) * sum_l S_l 2^(-8 (l - 2))
// (c < R: X = B^Q C_L, c >= R: Y = B^Q C_R).  A planes: rows ql * mp + m;
// B planes: rows c.  Each workgroup writes whole 1 KB row segments.
//
// With pm set, the tile also leaves the row maxima the exponents of X and Y
// need: for each of its rows m and each key (c / r) its columns meet, the
// largest |XY[ql][m][c]| over those columns, at
//     pm[((ql nct + cb) nslot + key - key0) mp + m]
// (cb = column tile, key0 = its first key, nslot >= the keys a tile meets).
// The tile's |XY| values go to LDS (the pipeline's buffers, free after the
// products), rows kPmLd doubles apart, and one thread per (row, key) takes the
// maximum over the key's columns.  The maximum is exact, so the exponents
// equal those of a pass over XY.
//
// The row and column exponents a lane needs (16 rows, 2 columns) are loaded
// before the products, so that their latency is hidden behind them.
constexpr int kPmLd = kNT + 1;      // LDS row stride of the |XY| tile (doubles)
static_assert(kHtMT * kPmLd * 8 <= PipeHt::LDS_BYTES, "|XY| tile in the pipeline's LDS");

__device__ __forceinline__ void ht_mixed_tile(const int8_t *__restrict__ Bp, i64 bpstride,
                                              i64 bkbstride, const int *__restrict__ eB,
                                              const int8_t *__restrict__ Cp, i64 cpstride,
                                              i64 ckbstride, const int *__restrict__ eC,
                                              double *__restrict__ XY, int nao, int R2, int mp,
                                              int cp, int nkb, int t, char *lds,
                                              double *__restrict__ pm = nullptr, int r = 1,
                                              int nslot = 0)
{
    typedef TileH TL;
    const int nmt = mp / kHtMT, nct = cp / kNT;
    const int ql = t / (nmt * nct), rem = t % (nmt * nct);
    const int mb = rem / nct, cb = rem % nct;
    // exponents of this lane's rows (element e of either tile) and columns
    // (rows < mp and columns < cp always have one)
    int eb[16], ec[kWTN];
#pragma unroll
    for (int e = 0; e < 16; e++) {
        int row, col;
        stile_coord_wide<TL>(0, e, row, col);
        eb[e] = eB[(i64)ql * mp + mb * kHtMT + row];
    }
#pragma unroll
    for (int tt = 0; tt < kWTN; tt++) {
        int row, col;
        stile_coord_wide<TL>(tt, 0, row, col);
        ec[tt] = eC[cb * kNT + col] + kSliceProdShift;
    }
    SPlanes a{Bp + (i64)ql * mp * kSliceKB, bpstride, bkbstride};
    SPlanes b{Cp, cpstride, ckbstride};
    SAccW<TL> acc;
    acc.zero();
    stile_gemm_w4<TL, kNS, kNbHt>(a, b, mb * kHtMT, cb * kNT, 0, nkb, lds, acc);
    double *out = XY + (i64)ql * nao * R2;
    double *tile = (double *)lds;
    if (pm)
        __syncthreads();                      // every wave past its last stage
#pragma unroll
    for (int tt = 0; tt < kWTN; tt++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
            int row, col;
            stile_coord_wide<TL>(tt, e, row, col);
            const int m = mb * kHtMT + row, c = cb * kNT + col;
            const double v = ldexp(combine_levels_wide<TL>(acc, tt, e), eb[e] + ec[tt]);
            if (m < nao && c < R2)
                out[(i64)m * R2 + c] = v;
            if (pm)
                tile[row * kPmLd + col] = fabs(v);
        }
    if (pm) {
        __syncthreads();
        const int c0 = cb * kNT, key0 = c0 / r;
        const int cend = (c0 + kNT) < R2 ? (c0 + kNT) : R2;
        double *dst = pm + (i64)(ql * nct + cb) * nslot * mp + mb * kHtMT;
        for (int e = threadIdx.x; e < kHtMT * nslot; e += TL::NTHR) {
            const int slot = e / kHtMT, row = e % kHtMT, key = key0 + slot;
            const int ca = key * r > c0 ? key * r - c0 : 0;
            const int cz = ((key + 1) * r < cend ? (key + 1) * r : cend) - c0;
            double mx = 0.0;
            for (int c = ca; c < cz; c++)
                mx = fmax(mx, tile[row * kPmLd + c]);
            dst[(i64)slot * mp + row] = mx;
        }
    }
}

__global__ void __launch_bounds__(256, 2) k_ht_mixed(const int8_t *__restrict__ Bp, i64 bpstride,
                                                     i64 bkbstride, const int *__restrict__ eB,
                                                     const int8_t *__restrict__ Cp, i64 cpstride,
                                                     i64 ckbstride, const int *__restrict__ eC,
                                                     double *__restrict__ XY, int nao, int R2, int mp,
                                                     int cp, int nkb, double *__restrict__ pm, int r,
                                                     int nslot)
{
    extern __shared__ char lds[];
    // consecutive tiles (the column tiles of a row panel) on one XCD, sharing its L2
    ht_mixed_tile(Bp, bpstride, bkbstride, eB, Cp, cpstride, ckbstride, eC, XY, nao, R2, mp, cp, nkb,
                  xcd_swizzle(blockIdx.x, gridDim.x), lds, pm, r, nslot);
}

// Partial-maximum slots per (row, column tile): the keys a column tile of
// kNT columns can meet.
__host__ __device__ inline int pm_slots(int r, int nkey)
{
    const int n = (kNT - 1) / r + 2;
    return n < nkey ? n : nkey;
}

// exps[key mpe + m] from the half-transform's partial maxima (rows of mp per
// slab, the half-transform's row pitch): the largest over the chunk's slabs
// and over the (one or two) column tiles that meet key's columns [key r,
// key r + r), for the 64 rows of row block mblk.  NW waves; wave w takes the
// slabs ql = w, w + NW, ... (coalesced 512-byte reads); the wave maxima meet
// in red.
template <int NW>
__device__ __forceinline__ void rowmax_pm_block(const double *__restrict__ pm, int nao, int nq,
                                                int nct, int mp, int mpe, int nslot, int r,
                                                int *__restrict__ exps, int mblk, int key,
                                                double (*red)[64])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = mblk * 64 + lane;
    const int mc = m < nao ? m : nao - 1;
    const int cb0 = key * r / kNT, cb1 = (key * r + r - 1) / kNT;
    const i64 qs = (i64)nct * nslot * mp;
    double mx = 0.0;
    for (int cb = cb0; cb <= cb1; cb++) {
        const int slot = key - cb * kNT / r;
        const double *p = pm + ((i64)cb * nslot + slot) * mp + mc;
        int ql = w;
        for (; ql + 3 * NW < nq; ql += 4 * NW) {
            const double v0 = p[(i64)ql * qs], v1 = p[(i64)(ql + NW) * qs];
            const double v2 = p[(i64)(ql + 2 * NW) * qs], v3 = p[(i64)(ql + 3 * NW) * qs];
            mx = fmax(mx, fmax(fmax(v0, v1), fmax(v2, v3)));
        }
        for (; ql < nq; ql += NW)
            mx = fmax(mx, p[(i64)ql * qs]);
    }
    red[w][lane] = mx;
    __syncthreads();
    if (w == 0 && m < nao) {
        double v = red[0][lane];
#pragma unroll
        for (int u = 1; u < NW; u++)
            v = fmax(v, red[u][lane]);
        exps[(i64)key * mpe + m] = row_exponent(v);
    }
}

// Workgroup: 64 rows of one key, 16 waves.
constexpr int kPmWaves = 16;
__global__ void __launch_bounds__(64 * kPmWaves) k_xy_rowmax_pm(const double *__restrict__ pm, int nao,
                                                               int nq, int nct, int mp, int mpe,
                                                               int nslot, int r,
                                                               int *__restrict__ exps)
{
    __shared__ double red[kPmWaves][64];
    rowmax_pm_block<kPmWaves>(pm, nao, nq, nct, mp, mpe, nslot, r, exps, blockIdx.x, blockIdx.y, red);
}

// ------------------------------------------------------------------ exchange
// Kp[s][k][m][n] (+)= scale 2^(eX + eY - 14) * sum_l S_l 2^(-8 (l - 2)) over the inner
// blocks [s * kbl, (s + 1) * kbl) of split s.  X/Y planes: rows k * mp + m
// from Xp / Yp (same strides); row exponents eX[k * mp + m], eY[k * mp + n].
__device__ __forceinline__ void ex_mixed_tile(const int8_t *__restrict__ Xp,
                                              const int8_t *__restrict__ Yp, i64 pstride,
                                              i64 kbstride, const int *__restrict__ eX,
                                              const int *__restrict__ eY, double *__restrict__ Kp,
                                              int nao, int nd, int mp, int nkb, int kbl,
                                              int accumulate, int sym, double scale, int t,
                                              char *lds)
{
    typedef TileS TL;
    const int nmt = mp / kMT, nnt = mp / kNT;
    // sym: Y = X, only the square tiles with nb >= mb (upper triangle)
    const int pk = sym ? nmt * (nmt + 1) / 2 : nmt * nnt;
    const int per = nd * pk;
    const int sp = t / per, rem0 = t % per;
    const int k = rem0 / pk, rem = rem0 % pk;
    int mb, nb;
    if (sym) {
        int q = rem;
        mb = 0;
        while (q >= nmt - mb) {
            q -= nmt - mb;
            mb++;
        }
        nb = mb + q;
    } else {
        mb = rem / nnt;
        nb = rem % nnt;
    }
    const int kb0 = sp * kbl < nkb ? sp * kbl : nkb;
    const int kb1 = (kb0 + kbl) < nkb ? (kb0 + kbl) : nkb;
    SPlanes a{Xp + (i64)k * mp * kSliceKB, pstride, kbstride};
    SPlanes b{Yp + (i64)k * mp * kSliceKB, pstride, kbstride};
    SAccW<TL> acc;
    acc.zero();
    stile_gemm_pp<TL, kNS, kNbEx>(a, b, mb * kMT, nb * kNT, kb0, kb1, lds, acc);
    double *Kk = Kp + ((i64)sp * nd + k) * nao * nao;
    // The lane's row and column exponents (rows and columns < mp all have
    // one), and per tile the partial sums it adds to, each loaded in one
    // batch so that their latencies overlap.
    int ex[16], ey[kWTN];
#pragma unroll
    for (int e = 0; e < 16; e++) {
        int row, col;
        stile_coord_wide<TL>(0, e, row, col);
        ex[e] = eX[(i64)k * mp + mb * kMT + row];
    }
#pragma unroll
    for (int tt = 0; tt < kWTN; tt++) {
        int row, col;
        stile_coord_wide<TL>(tt, 0, row, col);
        ey[tt] = eY[(i64)k * mp + nb * kNT + col] + kSliceProdShift;
    }
#pragma unroll
    for (int tt = 0; tt < kWTN; tt++) {
        double old[16];
#pragma unroll
        for (int e = 0; e < 16; e++) {
            int row, col;
            stile_coord_wide<TL>(tt, e, row, col);
            const int m = mb * kMT + row, n = nb * kNT + col;
            old[e] = (accumulate && m < nao && n < nao) ? Kk[(i64)m * nao + n] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 16; e++) {
            int row, col;
            stile_coord_wide<TL>(tt, e, row, col);
            const int m = mb * kMT + row, n = nb * kNT + col;
            if (m < nao && n < nao) {
                const double v = scale * ldexp(combine_levels_wide<TL>(acc, tt, e), ex[e] + ey[tt]);
                Kk[(i64)m * nao + n] = accumulate ? old[e] + v : v;
            }
        }
    }
}

__global__ void __launch_bounds__(512) k_ex_mixed(const int8_t *__restrict__ Xp,
                                                  const int8_t *__restrict__ Yp, i64 pstride,
                                                  i64 kbstride, const int *__restrict__ eX,
                                                  const int *__restrict__ eY,
                                                  double *__restrict__ Kp, int nao, int nd, int mp,
                                                  int nkb, int kbl, int accumulate, int sym,
                                                  double scale)
{
    extern __shared__ char lds[];
    ex_mixed_tile(Xp, Yp, pstride, kbstride, eX, eY, Kp, nao, nd, mp, nkb, kbl, accumulate, sym,
                  scale, xcd_swizzle(blockIdx.x, gridDim.x), lds);
}

// ------------------------------------------------------------------ batched
// The mixed phases over many members (jk_batched.hpp): the launch's table maps
// each workgroup to (member, tile); every member runs its own plan's chunk c
// with single-buffered planes, so a batched member is the same arithmetic as
// a single build of the same plan.

__global__ void __launch_bounds__(256) k_bm_slice_c(const BMember *__restrict__ M,
                                                    const int *__restrict__ tab)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    const i64 row = (i64)loc * 32 + (threadIdx.x >> 3);
    if (row >= m.cp)                 // whole 8-lane row groups leave together
        return;
    const int R2 = 2 * m.nd * m.r;
    slice_row8(m.Cc, 0, 1, R2, R2, m.nao, m.cp, m.kp / kSliceKB, m.Cp, m.cps, m.ckb, m.eC, row,
               threadIdx.x & 7);
}

template <int NJ>
__global__ void __launch_bounds__(256) k_bm_slice_b(const BMember *__restrict__ M,
                                                    const int *__restrict__ tab, int c)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    const i64 row = (i64)loc * 4 + (threadIdx.x >> 6);
    if (row >= (i64)nq * m.mpb)      // whole waves leave together
        return;
    slice_row_wave<NJ>(m.B + (i64)q0 * m.npos, m.npos, m.nao, m.nao, m.nao, m.mpb, m.kp / kSliceKB,
                       m.Bp, m.bps, m.bkb, m.eB, row);
}

// The chunk's packed slabs (jk.h JK_B_PACKED), bands of kBand rows; the
// dynamic LDS covers the largest member's band.
template <int NJ>
__global__ void __launch_bounds__(256) k_bm_slice_b_packed(const BMember *__restrict__ M,
                                                           const int *__restrict__ tab, int c)
{
    extern __shared__ double T[];
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    const int nband = (m.mpb + kBand - 1) / kBand;
    const int b = loc / nband, m0 = (loc % nband) * kBand;
    slice_band_packed<NJ>(m.B + (i64)(q0 + b) * m.bslab, b, m0, m.nao, m.mpb, m.kp / kSliceKB, m.Bp,
                          m.bps, m.bkb, m.eB, T);
}

__global__ void __launch_bounds__(256, 2) k_bm_ht(const BMember *__restrict__ M,
                                                  const int *__restrict__ tab, int c)
{
    extern __shared__ char lds[];
    int loc;
    const BMember &m = M[find_member(tab, xcd_local(blockIdx.x, gridDim.x), loc)];
    (void)c;
    const int nkey = m.sym ? m.nd : 2 * m.nd;
    ht_mixed_tile(m.Bp, m.bps, m.bkb, m.eB, m.Cp, m.cps, m.ckb, m.eC, m.XY, m.nao, nkey * m.r, m.mpb,
                  m.cpx, m.kp / kSliceKB, loc, lds, m.pm, m.r, pm_slots(m.r, nkey));
}

// Row exponents from the half-transform's partial maxima: tile loc of a
// member is (row block loc % nmb, key loc / nmb), 64 rows, four waves.
__global__ void __launch_bounds__(256) k_bm_rowmax(const BMember *__restrict__ M,
                                                   const int *__restrict__ tab, int c)
{
    __shared__ double red[4][64];
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    const int nkey = m.sym ? m.nd : 2 * m.nd, nmb = (m.nao + 63) / 64;
    rowmax_pm_block<4>(m.pm, m.nao, nq, m.cpx / kNT, m.mpb, m.mp, pm_slots(m.r, nkey), m.r, m.eXY,
                       loc % nmb, loc / nmb, red);
}

__global__ void __launch_bounds__(256) k_bm_slice_xy(const BMember *__restrict__ M,
                                                     const int *__restrict__ tab, int c)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    const int nkey = m.sym ? m.nd : 2 * m.nd;
    const int ngroup = cdiv_i((i64)nkey * m.mp, 32);
    const int row = (loc % ngroup) * 32 + (threadIdx.x >> 3);
    if (row >= nkey * m.mp)
        return;
    slice_xy_block(m.XY, m.nao, nkey, m.r, m.mp, nq * m.r, m.XYp, m.xps, m.xkb, m.eXY, row,
                   threadIdx.x & 7, loc / ngroup);
}

__global__ void __launch_bounds__(512) k_bm_ex(const BMember *__restrict__ M,
                                               const int *__restrict__ tab, int c)
{
    extern __shared__ char lds[];
    int loc;
    const BMember &m = M[find_member(tab, xcd_local(blockIdx.x, gridDim.x), loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    const int nkb = cdiv_i((i64)nq * m.r, kSliceKB);
    const int kbl = cdiv_i(nkb, m.nsplit);
    const int8_t *Xp = m.XYp, *Yp = m.sym ? Xp : m.XYp + (i64)m.nd * m.mp * kSliceKB;
    const int *eX = m.eXY, *eY = m.sym ? eX : m.eXY + (i64)m.nd * m.mp;
    ex_mixed_tile(Xp, Yp, m.xps, m.xkb, eX, eY, m.nsplit > 1 ? m.Kp : m.K, m.nao, m.nd, m.mp, nkb,
                  kbl, c > 0, m.sym, 1.0, loc, lds);
}

// ------------------------------------------------------------------ launchers
int mixed_nslice() { return kNS; }
int mixed_row_pad() { return kRowPad; }
int mixed_b_row_pad() { return kHtMT; }
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
                          int8_t *out, i64 pstride, i64 kbstride, int *exps, hipStream_t s)
{
    const int nj = cdiv(nkb, 8);
    if (nj > 8)     // long rows: generic two-pass slicer
        return launch_slice_rows(src, bs, rs, 1, nb, nr, nk, rp, nkb, out, pstride, kbstride, exps, s);
    const dim3 g(cdiv((i64)nb * rp, 4));
    {
        ProfScope ps_("slice_b", s);
        if (nj <= 1)
            hipLaunchKernelGGL(k_slice_rows_wave<1>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps);
        else if (nj <= 2)
            hipLaunchKernelGGL(k_slice_rows_wave<2>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps);
        else if (nj <= 4)
            hipLaunchKernelGGL(k_slice_rows_wave<4>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps);
        else
            hipLaunchKernelGGL(k_slice_rows_wave<8>, g, dim3(256), 0, s, src, bs, rs, nb, nr, nk, rp,
                               nkb, out, pstride, kbstride, exps);
    }
    return hipGetLastError();
}

// Dynamic LDS above 64 KB needs a per-kernel attribute, set once per
// (kernel, device).
static hipError_t set_lds(const void *fn, int bytes)
{
    static std::mutex mu;
    static std::set<std::pair<const void *, int>> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count({fn, dev}))
        return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        done.insert({fn, dev});
    return e;
}

hipError_t launch_slice_b_packed(const double *src, i64 bs, int nb, int nao, int rp, int nkb,
                                 int8_t *out, i64 pstride, i64 kbstride, int *exps, hipStream_t s)
{
    const int nj = cdiv(nkb, 8);
    if (nj > 8 || nao > rp)
        return hipErrorInvalidValue;        // rows beyond 2048 elements: not supported packed
    const dim3 g((unsigned)((i64)nb * cdiv(rp, kBand)));
    const size_t lds = sizeof(double) * kBand * nao;
    if (lds > 65536) {        // above 64 KB of dynamic LDS: per-kernel attribute
        const void *fn = nj <= 1   ? (const void *)k_slice_band_packed<1>
                         : nj <= 2 ? (const void *)k_slice_band_packed<2>
                         : nj <= 4 ? (const void *)k_slice_band_packed<4>
                                   : (const void *)k_slice_band_packed<8>;
        hipError_t e = set_lds(fn, (int)(sizeof(double) * kBand * 2048));
        if (e != hipSuccess)
            return e;
    }
    {
        ProfScope ps_("slice_b_packed", s);
        if (nj <= 1)
            hipLaunchKernelGGL(k_slice_band_packed<1>, g, dim3(256), lds, s, src, bs, nb, nao, rp,
                               nkb, out, pstride, kbstride, exps);
        else if (nj <= 2)
            hipLaunchKernelGGL(k_slice_band_packed<2>, g, dim3(256), lds, s, src, bs, nb, nao, rp,
                               nkb, out, pstride, kbstride, exps);
        else if (nj <= 4)
            hipLaunchKernelGGL(k_slice_band_packed<4>, g, dim3(256), lds, s, src, bs, nb, nao, rp,
                               nkb, out, pstride, kbstride, exps);
        else
            hipLaunchKernelGGL(k_slice_band_packed<8>, g, dim3(256), lds, s, src, bs, nb, nao, rp,
                               nkb, out, pstride, kbstride, exps);
    }
    return hipGetLastError();
}

// Packed slicer: rows of at most 2048 elements (and a band of 8 rows of
// LDS, 128 KB at that size).
int mixed_packed_ok(int nao, int kp) { return cdiv(kp / kSliceKB, 8) <= 8 && nao <= kp; }

int mixed_rowmax_ok(int R2) { return R2 <= 8192; }

hipError_t launch_slice_xy(const double *XY, int nao, int nkey, int r, int mp, int nj, int nkb,
                           int8_t *out, i64 pstride, i64 kbstride, const int *exps, hipStream_t s)
{
    {
        ProfScope ps_("slice_xy", s);
        hipLaunchKernelGGL(k_slice_xy, dim3(cdiv((i64)nkey * mp, 32), nkb < 65535 ? nkb : 65535),
                           dim3(256), 0, s, XY, nao, nkey, r, mp, nj, out, pstride, kbstride, exps,
                           nkb);
    }
    return hipGetLastError();
}


int xy_rowmax_slots(int r, int nkey) { return pm_slots(r, nkey); }

size_t xy_rowmax_pm_doubles(int nq, int mp, int cp, int r, int nkey)
{
    return (size_t)nq * (cp / kNT) * xy_rowmax_slots(r, nkey) * mp;
}

hipError_t launch_ht_mixed(const int8_t *Bp, i64 bpstride, i64 bkbstride, const int *eB,
                           const int8_t *Cp, i64 cpstride, i64 ckbstride, const int *eC, double *XY,
                           int nao, int R2, int nq, int mp, int cp, int nkb, hipStream_t s,
                           double *pm, int r)
{
    hipError_t e = set_lds((const void *)k_ht_mixed, PipeHt::LDS_BYTES);
    if (e != hipSuccess)
        return e;
    const int nslot = pm ? xy_rowmax_slots(r, R2 / r) : 0;
    if (pm && (size_t)kHtMT * nslot * sizeof(double) > (size_t)PipeHt::LDS_BYTES)
        return hipErrorInvalidValue;
    {
        ProfScope ps_("ht_mixed", s);
        hipLaunchKernelGGL(k_ht_mixed, dim3(nq * (mp / kHtMT) * (cp / kNT)), dim3(TileH::NTHR),
                           PipeHt::LDS_BYTES, s, Bp, bpstride, bkbstride, eB, Cp, cpstride, ckbstride,
                           eC, XY, nao, R2, mp, cp, nkb, pm, r, nslot);
    }
    return hipGetLastError();
}

hipError_t launch_xy_rowmax_pm(const double *pm, int nao, int nq, int nkey, int r, int mp, int mpe,
                               int cp, int *exps, hipStream_t s)
{
    {
        ProfScope ps_("xy_rowmax_pm", s);
        hipLaunchKernelGGL(k_xy_rowmax_pm, dim3(cdiv(nao, 64), nkey), dim3(64 * kPmWaves), 0, s, pm, nao, nq,
                           cp / kNT, mp, mpe, xy_rowmax_slots(r, nkey), r, exps);
    }
    return hipGetLastError();
}

int mixed_max_depth() { return kSliceMaxDepth; }

int ex_mixed_nsplit(int mp, int nd, int nkb, int sym)
{
    // one 512-thread workgroup per CU (registers), so half the usual slots
    const int nmt = mp / kMT;
    const int tiles = nd * (sym ? nmt * (nmt + 1) / 2 : nmt * (mp / kNT));
    int maxs = nkb / 16 > 1 ? nkb / 16 : 1;
    if (maxs > 16)
        maxs = 16;
    const int s = pick_split_slots(tiles, maxs, device_slots() / 2);
    // exact int32 level sums: a split of cdiv(nkb, s) inner blocks may hold at
    // most kSliceMaxDepth inner indices
    const int need = cdiv(nkb, kSliceMaxDepth / kSliceKB);
    return s > need ? s : need;
}

hipError_t launch_ex_mixed(const int8_t *Xp, const int8_t *Yp, i64 pstride, i64 kbstride,
                           const int *eX, const int *eY, double *Kp, int nao, int nd, int mp, int nkb,
                           int nsplit, int accumulate, hipStream_t s, int sym, double scale)
{
    hipError_t e = set_lds((const void *)k_ex_mixed, PipeEx::LDS_BYTES);
    if (e != hipSuccess)
        return e;
    const int kbl = cdiv(nkb, nsplit);
    const int nmt = mp / kMT;
    const int pk = sym ? nmt * (nmt + 1) / 2 : nmt * (mp / kNT);
    {
        ProfScope ps_("ex_mixed", s);
        hipLaunchKernelGGL(k_ex_mixed, dim3(nsplit * nd * pk), dim3(TileS::NTHR), PipeEx::LDS_BYTES, s, Xp,
                           Yp, pstride, kbstride, eX, eY, Kp, nao, nd, mp, nkb, kbl, accumulate, sym,
                           scale);
    }
    return hipGetLastError();
}

// Dynamic LDS of the batched mixed kernels above 64 KB, set once per device
// before a launch sequence is captured.
hipError_t prepare_batched_mixed_kernels()
{
    hipError_t e = set_lds((const void *)k_bm_ht, PipeHt::LDS_BYTES);
    if (e == hipSuccess)
        e = set_lds((const void *)k_bm_ex, PipeEx::LDS_BYTES);
    // the packed slicer's band of the longest rows the packed path takes
    const int band = (int)sizeof(double) * kBand * 2048;
    if (e == hipSuccess)
        e = set_lds((const void *)k_bm_slice_b_packed<1>, band);
    if (e == hipSuccess)
        e = set_lds((const void *)k_bm_slice_b_packed<2>, band);
    if (e == hipSuccess)
        e = set_lds((const void *)k_bm_slice_b_packed<4>, band);
    if (e == hipSuccess)
        e = set_lds((const void *)k_bm_slice_b_packed<8>, band);
    return e;
}

hipError_t launch_batched_mixed_phase(int phase, const BMember *M, const int *tab, int ntiles,
                                      int step, hipStream_t s, int arg)
{
    const dim3 g(ntiles);
    switch (phase) {
    case kPhaseMSliceC: {
        ProfScope ps_("bm_slice_c", s);
        hipLaunchKernelGGL(k_bm_slice_c, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseMSliceB: {
        ProfScope ps_("bm_slice_b", s);
        if (arg <= 1)
            hipLaunchKernelGGL(k_bm_slice_b<1>, g, dim3(256), 0, s, M, tab, step);
        else if (arg <= 2)
            hipLaunchKernelGGL(k_bm_slice_b<2>, g, dim3(256), 0, s, M, tab, step);
        else if (arg <= 4)
            hipLaunchKernelGGL(k_bm_slice_b<4>, g, dim3(256), 0, s, M, tab, step);
        else if (arg <= 8)
            hipLaunchKernelGGL(k_bm_slice_b<8>, g, dim3(256), 0, s, M, tab, step);
        else
            return hipErrorInvalidValue;
        break;
    }
    case kPhaseMSliceBPacked: {
        // arg = 16 x (dynamic LDS bytes) + register blocks
        const int nj = arg & 15;
        const size_t lds = (size_t)(arg >> 4);
        if (lds > sizeof(double) * kBand * 2048)
            return hipErrorInvalidValue;
        ProfScope ps_("bm_slice_b_packed", s);
        if (nj <= 1)
            hipLaunchKernelGGL(k_bm_slice_b_packed<1>, g, dim3(256), lds, s, M, tab, step);
        else if (nj <= 2)
            hipLaunchKernelGGL(k_bm_slice_b_packed<2>, g, dim3(256), lds, s, M, tab, step);
        else if (nj <= 4)
            hipLaunchKernelGGL(k_bm_slice_b_packed<4>, g, dim3(256), lds, s, M, tab, step);
        else if (nj <= 8)
            hipLaunchKernelGGL(k_bm_slice_b_packed<8>, g, dim3(256), lds, s, M, tab, step);
        else
            return hipErrorInvalidValue;
        break;
    }
    case kPhaseMHalf: {
        ProfScope ps_("bm_ht_mixed", s);
        hipLaunchKernelGGL(k_bm_ht, g, dim3(TileH::NTHR), PipeHt::LDS_BYTES, s, M, tab, step);
        break;
    }
    case kPhaseMRowmax: {
        ProfScope ps_("bm_xy_rowmax", s);
        hipLaunchKernelGGL(k_bm_rowmax, g, dim3(256), 0, s, M, tab, step);
        break;
    }
    case kPhaseMSliceXY: {
        ProfScope ps_("bm_slice_xy", s);
        hipLaunchKernelGGL(k_bm_slice_xy, g, dim3(256), 0, s, M, tab, step);
        break;
    }
    case kPhaseMExchange: {
        ProfScope ps_("bm_ex_mixed", s);
        hipLaunchKernelGGL(k_bm_ex, g, dim3(TileS::NTHR), PipeEx::LDS_BYTES, s, M, tab, step);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Tile counts of the batched mixed phases for one member (host).
int mixed_ht_tiles(int mp, int cpx, int nq) { return nq * (mp / kHtMT) * (cpx / kNT); }
int mixed_ex_tiles(int mp, int nd, int nsplit, int sym)
{
    const int nmt = mp / kMT;
    return nsplit * nd * (sym ? nmt * (nmt + 1) / 2 : nmt * (mp / kNT));
}

} // namespace jk
