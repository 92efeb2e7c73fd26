// jk_fp64.hip -- single-problem FP64 kernels of the Cholesky-decomposed J/K
// build: each kernel runs tile blockIdx.x of one phase (jk_tiles.hpp).
#include "jk_kernels.hpp"
#include "jk_tiles.hpp"

#include <mutex>
#include <set>
#include <utility>

namespace jk {

__global__ void __launch_bounds__(256) k_pack_c(const double *__restrict__ CL,
                                                const double *__restrict__ CR, double *__restrict__ Cc,
                                                int nao, int nd, int r)
{
    pack_tile(CL, CR, Cc, nao, nd, r, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_density(const double *__restrict__ CL,
                                                 const double *__restrict__ CR, double *__restrict__ D,
                                                 int nao, int r)
{
    __shared__ double lds[TileDensity::LDS_DOUBLES];
    density_tile(CL, CR, D, nao, r, blockIdx.x, lds);
}

__global__ void __launch_bounds__(256) k_project(const double *__restrict__ B,
                                                 const double *__restrict__ A, double *__restrict__ part,
                                                 int naux, int nd, i64 npos, int plen)
{
    __shared__ double lds[TileProject::LDS_DOUBLES];
    project_tile(B, A, part, naux, nd, npos, plen, blockIdx.x, lds);
}

__global__ void __launch_bounds__(256) k_project16(const double *__restrict__ B,
                                                   const double *__restrict__ A,
                                                   double *__restrict__ part, int naux, int nd,
                                                   i64 npos, int plen)
{
    __shared__ double lds[TileProject16::LDS_DOUBLES];
    project16_tile(B, A, part, naux, nd, npos, plen, blockIdx.x, lds);
}

__global__ void __launch_bounds__(256) k_project_reduce(const double *__restrict__ part,
                                                        double *__restrict__ g, int naux, int nd,
                                                        int npb)
{
    reduce_tile(part, g, naux, nd, npb, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_coulomb(const double *__restrict__ B,
                                                 const double *__restrict__ g, double *__restrict__ J,
                                                 int naux, int nd, i64 npos, double scale,
                                                 int accumulate)
{
    coulomb_tile(B, g, J, naux, nd, npos, blockIdx.x, scale, accumulate);
}

__global__ void __launch_bounds__(256, 3) k_half_transform(const double *__restrict__ B,
                                                           const double *__restrict__ Cc,
                                                           double *__restrict__ Xw,
                                                           double *__restrict__ Yw, int nao, int nd,
                                                           int r, int q0, int nq, int ldw, int ncol)
{
    __shared__ double lds[TileHalf::LDS_DOUBLES];
    const int n = ht_tiles_cols(nao, ncol, nq);
    ht_tile(B, Cc, Xw, Yw, nao, nd, r, q0, ldw, xcd_swizzle(blockIdx.x, n), lds, ncol);
}

// The half-transform with 64 x 64 tiles (four workgroups per CU): a plan
// choice (jk_tune.h) for shapes where the 128-row tiles waste rows.
__global__ void __launch_bounds__(256, 4) k_half_transform64(const double *__restrict__ B,
                                                             const double *__restrict__ Cc,
                                                             double *__restrict__ Xw,
                                                             double *__restrict__ Yw, int nao,
                                                             int nd, int r, int q0, int nq, int ldw,
                                                             int ncol)
{
    __shared__ double lds[TileHalf64::LDS_DOUBLES];
    const int n = nq * cdiv_i(nao, 64) * cdiv_i(ncol, 64);
    ht_tile_tl<TileHalf64>(B, Cc, Xw, Yw, nao, nd, r, q0, ldw, xcd_swizzle(blockIdx.x, n), lds,
                           ncol);
}

// The half-transform with the 128 x 64 tile split over eight 64 x 16 wave
// tiles (110 VGPRs, four waves per SIMD): more waves to hide the fragment
// reads and barriers of each stage (measured 49.7 against 47.3 TF at nao 500).
typedef Tile<128, 64, 64, 16, 16> TileHalfW8;
__global__ void __launch_bounds__(512, 2) k_half_transform_w8(const double *__restrict__ B,
                                                              const double *__restrict__ Cc,
                                                              double *__restrict__ Xw,
                                                              double *__restrict__ Yw, int nao,
                                                              int nd, int r, int q0, int nq,
                                                              int ldw, int ncol)
{
    __shared__ double lds[TileHalfW8::LDS_DOUBLES];
    const int n = ht_tiles_cols(nao, ncol, nq);
    ht_tile_tl<TileHalfW8>(B, Cc, Xw, Yw, nao, nd, r, q0, ldw, xcd_swizzle(blockIdx.x, n), lds,
                           ncol);
}

// The half-transform on the 16 x 16 x 4 engine, over the chunk's stacked
// slabs: 128 x 128 tiles of four 64 x 64 wave tiles in stages of 8 inner
// indices (two workgroups per CU), or 128 x 64 tiles of four 64 x 32 wave
// tiles in stages of 16 (three workgroups per CU).  Dynamic LDS: 35 and 52 KB.
typedef Tile16<128, 128, 64, 64, 8> TileH16a;
typedef TileHalf16 TileH16c;
__global__ void __launch_bounds__(256, 2) k_half_transform16a(const double *__restrict__ B,
                                                              const double *__restrict__ Cc,
                                                              double *__restrict__ Xw,
                                                              double *__restrict__ Yw, int nao,
                                                              int nd, int r, int q0, int nq,
                                                              int ldw, int ncol)
{
    extern __shared__ double lds_dyn[];
    const int n = ht_flat_tiles<TileH16a>(nao, ncol, nq);
    ht_tile_flat<TileH16a>(B, Cc, Xw, Yw, nao, nd, r, q0, nq, ldw, xcd_swizzle(blockIdx.x, n),
                           lds_dyn, ncol);
}
__global__ void __launch_bounds__(256, 3) k_half_transform16(const double *__restrict__ B,
                                                             const double *__restrict__ Cc,
                                                             double *__restrict__ Xw,
                                                             double *__restrict__ Yw, int nao,
                                                             int nd, int r, int q0, int nq, int ldw,
                                                             int ncol)
{
    extern __shared__ double lds_dyn[];
    const int n = ht_flat_tiles<TileH16c>(nao, ncol, nq);
    ht_tile_flat<TileH16c>(B, Cc, Xw, Yw, nao, nd, r, q0, nq, ldw, xcd_swizzle(blockIdx.x, n),
                           lds_dyn, ncol);
}

// Packed slabs on the 16 x 16 x 4 engine (plan tiles 3 and 4): 128 x 64 tiles
// per slab, three workgroups per CU.
__global__ void __launch_bounds__(256, 3) k_half_transform16_packed(const double *__restrict__ B,
                                                                    const double *__restrict__ Cc,
                                                                    double *__restrict__ Xw,
                                                                    double *__restrict__ Yw,
                                                                    int nao, int nd, int r, int q0,
                                                                    int nq, int ldw, int ncol)
{
    extern __shared__ double lds_dyn[];
    const int n = nq * cdiv_i(nao, TileHalf16::BM) * cdiv_i(ncol, TileHalf16::BN);
    ht_tile16_packed<TileHalf16>(B, Cc, Xw, Yw, nao, nd, r, q0, ldw, xcd_swizzle(blockIdx.x, n),
                                 lds_dyn, ncol);
}

// The same on packed slabs (jk.h JK_B_PACKED).
__global__ void __launch_bounds__(256, 3) k_half_transform_packed(const double *__restrict__ B,
                                                                  const double *__restrict__ Cc,
                                                                  double *__restrict__ Xw,
                                                                  double *__restrict__ Yw, int nao,
                                                                  int nd, int r, int q0, int nq,
                                                                  int ldw, int ncol)
{
    __shared__ double lds[TileHalf::LDS_DOUBLES];
    const int n = ht_tiles_cols(nao, ncol, nq);
    ht_tile<true>(B, Cc, Xw, Yw, nao, nd, r, q0, ldw, xcd_swizzle(blockIdx.x, n), lds, ncol);
}

// S_k packed from D_k: S[m <= n] = D[m][n] + D[n][m] (m < n), D[m][m], so
// that <B^Q, D_k> = sum over the packed positions of B^Q S_k.  Block (k, m).
__global__ void __launch_bounds__(256) k_sym_pack(const double *__restrict__ D,
                                                  double *__restrict__ S, int nao)
{
    const int k = blockIdx.x, m = blockIdx.y;
    const double *Dk = D + (i64)k * nao * nao;
    double *Sk = S + (i64)k * pk_size(nao) + pk_row(m, nao) - m;
    for (int n = m + threadIdx.x; n < nao; n += 256)
        Sk[n] = n == m ? Dk[(i64)m * nao + m] : Dk[(i64)m * nao + n] + Dk[(i64)n * nao + m];
}

// out[k][m][n] (+)= scale * P[k][(m, n)] for packed symmetric P.  Block (k, m).
__global__ void __launch_bounds__(256) k_unpack_sym(const double *__restrict__ P,
                                                    double *__restrict__ out, int nao, double scale,
                                                    int accumulate)
{
    const int k = blockIdx.x, m = blockIdx.y;
    const double *Pk = P + (i64)k * pk_size(nao);
    double *o = out + ((i64)k * nao + m) * nao;
    for (int n = threadIdx.x; n < nao; n += 256) {
        const double v = scale * Pk[pk_index(m, n, nao)];
        o[n] = accumulate ? o[n] + v : v;
    }
}

// The exchange product on the 16 x 16 x 4 engine: the same 128 x 64 tiles,
// four 64 x 32 wave tiles, three workgroups per CU (52 KB of dynamic LDS).
typedef TileH16c TileEx16;
template <bool MASK>
__global__ void __launch_bounds__(256, 3) k_exchange16(const double *__restrict__ Xw,
                                                       const double *__restrict__ Yw,
                                                       double *__restrict__ Kp, int nao, int nd,
                                                       int nj, int ldw, int nsplit, int jlen,
                                                       int accumulate, int sym, double scale)
{
    extern __shared__ double lds_dyn[];
    const int n = nsplit * nd * (sym ? ex_tri_tiles(nao) : cdiv_i(nao, kExM) * cdiv_i(nao, kExN));
    ex_tile<TileEx16, MASK>(Xw, Yw, Kp, nao, nd, nj, ldw, jlen, accumulate,
                            xcd_swizzle(blockIdx.x, n), lds_dyn, sym, scale);
}

__global__ void __launch_bounds__(512, 4) k_exchange(const double *__restrict__ Xw,
                                                     const double *__restrict__ Yw,
                                                     double *__restrict__ Kp, int nao, int nd, int nj,
                                                     int ldw, int nsplit, int jlen, int accumulate,
                                                     int sym, double scale)
{
    __shared__ double lds[TileExch::LDS_DOUBLES];
    const int n = nsplit * nd * (sym ? ex_tri_tiles(nao) : cdiv_i(nao, kExM) * cdiv_i(nao, kExN));
    ex_tile(Xw, Yw, Kp, nao, nd, nj, ldw, jlen, accumulate, xcd_swizzle(blockIdx.x, n), lds, sym,
            scale);
}

__global__ void __launch_bounds__(256) k_mirror_upper(double *__restrict__ K, int nao, int nd)
{
    __shared__ double t[32][33];
    // densities k = blockIdx.y, + gridDim.y, ... (grid y is capped at 65535)
    for (int k = blockIdx.y; k < nd; k += gridDim.y)
        mirror_tile(K + (i64)k * nao * nao, nao, blockIdx.x, t);
}

__global__ void __launch_bounds__(256) k_sum_splits(const double *__restrict__ part,
                                                    double *__restrict__ out, i64 n, int nsplit)
{
    sum_tile(part, out, n, nsplit, blockIdx.x);
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

int pick_split(int tiles, int smax) { return pick_split_slots(tiles, smax, device_slots()); }

int pick_split_slots(int tiles, int smax, int slots)
{
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
    {
        ProfScope ps_("pack_c", s);
        hipLaunchKernelGGL(k_pack_c, dim3(pack_tiles(nao, nd, r)), dim3(256), 0, s, CL, CR, Cc, nao,
                           nd, r);
    }
    return hipGetLastError();
}

hipError_t launch_density(const double *CL, const double *CR, double *D, int nao, int nd, int r,
                          hipStream_t s)
{
    {
        ProfScope ps_("density", s);
        hipLaunchKernelGGL(k_density, dim3(density_tiles(nao, nd)), dim3(256), 0, s, CL, CR, D, nao, r);
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
    {
        ProfScope ps_("project", s);
        hipLaunchKernelGGL(k_project, dim3(project_tiles(naux, nd, npb)), dim3(256), 0, s, B, A, part,
                           naux, nd, npos, plen);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("project_reduce", s);
        hipLaunchKernelGGL(k_project_reduce, dim3(reduce_tiles(naux, nd)), dim3(256), 0, s, part, g,
                           naux, nd, npb);
    }
    return hipGetLastError();
}

int project16_nblocks(i64 npos, int naux, int *plen) { return project_nblocks(npos, naux, 8, plen); }

hipError_t launch_project16(const double *B, const double *A, double *part, double *g, int naux,
                            int nd, i64 npos, hipStream_t s)
{
    if (nd <= 8 || nd > 16)
        return hipErrorInvalidValue;
    int plen;
    const int npb = project16_nblocks(npos, naux, &plen);
    {
        ProfScope ps_("project16", s);
        hipLaunchKernelGGL(k_project16, dim3(project16_tiles(naux, npb)), dim3(256), 0, s, B, A,
                           part, naux, nd, npos, plen);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("project_reduce", s);
        hipLaunchKernelGGL(k_project_reduce, dim3(reduce_tiles(naux, nd)), dim3(256), 0, s, part, g,
                           naux, nd, npb);
    }
    return hipGetLastError();
}

hipError_t launch_coulomb(const double *B, const double *g, double *J, int naux, int nd, i64 npos,
                          hipStream_t s, double scale, int accumulate)
{
    {
        ProfScope ps_("coulomb", s);
        hipLaunchKernelGGL(k_coulomb, dim3(coulomb_tiles(nd, npos)), dim3(256), 0, s, B, g, J, naux, nd,
                           npos, scale, accumulate);
    }
    return hipGetLastError();
}

// Dynamic LDS above 64 KB needs a per-kernel attribute, set once per
// (kernel, device).
hipError_t set_dynamic_lds(const void *fn, int bytes)
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

hipError_t launch_half_transform(const double *B, const double *Cc, double *Xw, double *Yw,
                                 int nao, int nd, int r, int q0, int nq, int ldw, hipStream_t s,
                                 int ncol, int packed, int tile, const char *prof)
{
    if (ncol < 0)
        ncol = 2 * nd * r;
    // packed slabs: one buffer resource per slab
    if (!packed && tile >= 3 && !buf_extent_ok((i64)nq * nao * nao))
        tile = 2;                                 // chunk beyond the buffer loads' 4 GiB reach
    if (packed && tile >= 3) {
        const int lds = (int)sizeof(double) * TileHalf16::LDS_DOUBLES;
        hipError_t e = set_dynamic_lds((const void *)k_half_transform16_packed, lds);
        if (e != hipSuccess)
            return e;
        ProfScope ps_("half_transform_packed", s);
        hipLaunchKernelGGL(k_half_transform16_packed,
                           dim3(nq * cdiv(nao, TileHalf16::BM) * cdiv(ncol, TileHalf16::BN)),
                           dim3(TileHalf16::NTHR), lds, s, B, Cc, Xw, Yw, nao, nd, r, q0, nq, ldw,
                           ncol);
    } else if (packed) {
        ProfScope ps_("half_transform_packed", s);
        hipLaunchKernelGGL(k_half_transform_packed, dim3(ht_tiles_cols(nao, ncol, nq)), dim3(256), 0,
                           s, B, Cc, Xw, Yw, nao, nd, r, q0, nq, ldw, ncol);
    } else if (tile == 3 || tile == 4) {
        const void *fn = tile == 3 ? (const void *)k_half_transform16a : (const void *)k_half_transform16;
        const int lds = (int)sizeof(double) * (tile == 3 ? TileH16a::LDS_DOUBLES : TileH16c::LDS_DOUBLES);
        hipError_t e = set_dynamic_lds(fn, lds);
        if (e != hipSuccess)
            return e;
        ProfScope ps_(prof, s);
        if (tile == 3)
            hipLaunchKernelGGL(k_half_transform16a, dim3(ht_flat_tiles<TileH16a>(nao, ncol, nq)),
                               dim3(256), lds, s, B, Cc, Xw, Yw, nao, nd, r, q0, nq, ldw, ncol);
        else
            hipLaunchKernelGGL(k_half_transform16, dim3(ht_flat_tiles<TileH16c>(nao, ncol, nq)),
                               dim3(256), lds, s, B, Cc, Xw, Yw, nao, nd, r, q0, nq, ldw, ncol);
    } else if (tile == 2) {
        ProfScope ps_(prof, s);
        hipLaunchKernelGGL(k_half_transform_w8, dim3(ht_tiles_cols(nao, ncol, nq)), dim3(512), 0, s, B,
                           Cc, Xw, Yw, nao, nd, r, q0, nq, ldw, ncol);
    } else if (tile == 1) {
        ProfScope ps_(prof, s);
        hipLaunchKernelGGL(k_half_transform64, dim3(nq * cdiv(nao, 64) * cdiv(ncol, 64)), dim3(256), 0,
                           s, B, Cc, Xw, Yw, nao, nd, r, q0, nq, ldw, ncol);
    } else {
        ProfScope ps_(prof, s);
        hipLaunchKernelGGL(k_half_transform, dim3(ht_tiles_cols(nao, ncol, nq)), dim3(256), 0, s, B, Cc,
                           Xw, Yw, nao, nd, r, q0, nq, ldw, ncol);
    }
    return hipGetLastError();
}

hipError_t launch_sym_pack(const double *D, double *S, int nao, int nd, hipStream_t s)
{
    {
        ProfScope ps_("sym_pack", s);
        hipLaunchKernelGGL(k_sym_pack, dim3(nd, nao), dim3(256), 0, s, D, S, nao);
    }
    return hipGetLastError();
}

hipError_t launch_unpack_sym(const double *P, double *out, int nao, int nd, double scale,
                             int accumulate, hipStream_t s)
{
    {
        ProfScope ps_("unpack_sym", s);
        hipLaunchKernelGGL(k_unpack_sym, dim3(nd, nao), dim3(256), 0, s, P, out, nao, scale,
                           accumulate);
    }
    return hipGetLastError();
}

hipError_t launch_mirror_upper(double *K, int nao, int nd, hipStream_t s)
{
    const int nb = cdiv(nao, 32);
    {
        ProfScope ps_("mirror", s);
        hipLaunchKernelGGL(k_mirror_upper, dim3(nb * (nb + 1) / 2, nd < 65535 ? nd : 65535), dim3(256),
                           0, s, K, nao, nd);
    }
    return hipGetLastError();
}

int exchange_nsplit(int nao, int nd, int nj, int sym)
{
    // Full rounds of workgroups; each split keeps >= 256 inner indices.
    const int tiles = nd * (sym ? ex_tri_tiles(nao) : cdiv(nao, kExM) * cdiv(nao, kExN));
    int maxs = nj / 256 > 1 ? nj / 256 : 1;
    if (maxs > 16)
        maxs = 16;
    // k_exchange16 holds three workgroups per CU
    return pick_split_slots(tiles, maxs, device_slots() / 2 * 3);
}

hipError_t launch_exchange(const double *Xw, const double *Yw, double *Kp, int nao, int nd, int nj,
                           int ldw, int nsplit, int accumulate, hipStream_t s, int sym, double scale)
{
    int jlen = cdiv(nj, nsplit);
    jlen = ((jlen + 15) / 16) * 16;
    const int per = sym ? ex_tri_tiles(nao) : cdiv(nao, kExM) * cdiv(nao, kExN);
    if (buf_extent_ok((i64)nao * ldw)) {
        // splits end on 16-deep stage boundaries (jlen is a multiple of 16), so
        // only a depth nj off that grid leaves a stage to mask
        const bool mask = nj % 16 != 0;
        const int lds = (int)sizeof(double) * TileEx16::LDS_DOUBLES;
        hipError_t e = set_dynamic_lds(mask ? (const void *)k_exchange16<true>
                                            : (const void *)k_exchange16<false>, lds);
        if (e != hipSuccess)
            return e;
        ProfScope ps_("exchange", s);
        if (mask)
            hipLaunchKernelGGL(k_exchange16<true>, dim3(nsplit * nd * per), dim3(TileEx16::NTHR), lds,
                               s, Xw, Yw, Kp, nao, nd, nj, ldw, nsplit, jlen, accumulate, sym, scale);
        else
            hipLaunchKernelGGL(k_exchange16<false>, dim3(nsplit * nd * per), dim3(TileEx16::NTHR), lds,
                               s, Xw, Yw, Kp, nao, nd, nj, ldw, nsplit, jlen, accumulate, sym, scale);
    } else {
        ProfScope ps_("exchange", s);
        hipLaunchKernelGGL(k_exchange, dim3(nsplit * nd * per), dim3(TileExch::NTHR), 0, s, Xw, Yw, Kp,
                           nao, nd, nj, ldw, nsplit, jlen, accumulate, sym, scale);
    }
    return hipGetLastError();
}

hipError_t launch_sum_splits(const double *part, double *out, i64 n, int nsplit, hipStream_t s)
{
    {
        ProfScope ps_("sum_splits", s);
        hipLaunchKernelGGL(k_sum_splits, dim3(sum_tiles(n)), dim3(256), 0, s, part, out, n, nsplit);
    }
    return hipGetLastError();
}

} // namespace jk
