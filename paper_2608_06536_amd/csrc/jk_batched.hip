// jk_batched.hip -- many J/K problems of uneven size per launch.
//
// A batched build runs the phases of the FP64 build (jk_tiles.hpp) once for
// the whole batch: each launch covers the tiles of every member that takes
// part in that phase, in one grid.  blockIdx.x is mapped to (member, tile)
// through a table of prefix sums; members are listed in decreasing order of
// per-tile cost so the longest tiles start first.  Each member runs the
// single-build plan for a chunk budget of 256 MB (members own their chunk
// buffers, so the budget is smaller than a single build's 1 GB); where both
// budgets give the same chunking -- every problem whose slabs fit one 256 MB
// chunk -- its outputs are bit-for-bit those of a single jk_build.
//
// The member descriptors and the tables live in the caller's workspace; the
// host writes them with one asynchronous copy per call.  Kernel arguments are
// only workspace pointers, so a captured graph of the launch sequence can be
// replayed for any batch of the same shapes in the same workspace.
#include "jk_batched.hpp"
#include "jk_kernels.hpp"
#include "jk_tiles.hpp"
#include "coulomb_upper.hpp"

namespace jk {

__global__ void __launch_bounds__(256) k_b_pack(const BMember *__restrict__ M, const int *__restrict__ tab)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    pack_tile(m.CL, m.CR, m.Cc, m.nao, m.nd, m.r, loc);
}

__global__ void __launch_bounds__(256) k_b_density(const BMember *__restrict__ M,
                                                   const int *__restrict__ tab)
{
    __shared__ double lds[TileDensity::LDS_DOUBLES];
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    density_tile(m.CL, m.CR, m.D, m.nao, m.r, loc, lds);
}

// S_k = D_k + D_k^T on the packed positions (D_k[m][m] on the diagonal):
// one row m of one k per workgroup.
__global__ void __launch_bounds__(256) k_b_sym_pack(const BMember *__restrict__ M,
                                                    const int *__restrict__ tab)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    const int k = loc / m.nao, a = loc % m.nao;
    const double *Dk = m.D + (i64)k * m.npos;
    double *row = m.S + (i64)k * m.bslab + pk_row(a, m.nao) - a;
    for (int b = a + threadIdx.x; b < m.nao; b += 256)
        row[b] = b == a ? Dk[(i64)a * m.nao + a] : Dk[(i64)a * m.nao + b] + Dk[(i64)b * m.nao + a];
}

// D_k folded onto its upper triangle in place (coulomb_upper.hpp): one row
// per workgroup.
__global__ void __launch_bounds__(256) k_b_fold_upper(const BMember *__restrict__ M,
                                                      const int *__restrict__ tab)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    fold_upper_row(m.D, m.nao, loc / m.nao, loc % m.nao);
}

// J_k[a][b] from the packed J_k the Coulomb phase left in D: one row per
// workgroup.
__global__ void __launch_bounds__(256) k_b_unpack_j(const BMember *__restrict__ M,
                                                    const int *__restrict__ tab)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    const int k = loc / m.nao, a = loc % m.nao;
    const double *Pk = m.D + (i64)k * m.bslab;
    double *o = m.J + ((i64)k * m.nao + a) * m.nao;
    for (int b = threadIdx.x; b < m.nao; b += 256)
        o[b] = Pk[pk_index(a, b, m.nao)];
}

__global__ void __launch_bounds__(256) k_b_project(const BMember *__restrict__ M,
                                                   const int *__restrict__ tab)
{
    __shared__ double lds[TileProject::LDS_DOUBLES];
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    if (m.packed)
        project_tile(m.B, m.S, m.part, m.naux, m.nd, m.bslab, m.plen, loc, lds);
    else
        project_upper_tile<TileProject, 8>(m.B, m.D, m.part, m.naux, m.nd, m.nao, m.plen, loc, lds);
}

__global__ void __launch_bounds__(256) k_b_reduce(const BMember *__restrict__ M,
                                                  const int *__restrict__ tab)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    reduce_tile(m.part, m.g, m.naux, m.nd, m.npb, loc);
}

// ws: the workspace start (where M lies), as doubles; g is read at ws + goff.
__global__ void __launch_bounds__(256) k_b_coulomb(const BMember *__restrict__ M,
                                                   const int *__restrict__ tab,
                                                   const double *__restrict__ ws)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    const double *g = ws + m.goff;
    if (m.packed)
        coulomb_tile(m.B, g, m.D, m.naux, m.nd, m.bslab, loc);
    else
        coulomb_upper_tile(m.B, g, m.J, m.nao, m.naux, m.nd, loc);
}

__global__ void __launch_bounds__(256, 3) k_b_half_transform(const BMember *__restrict__ M,
                                                             const int *__restrict__ tab, int c)
{
    __shared__ double lds[TileHalf::LDS_DOUBLES];
    int loc;
    const BMember &m = M[find_member(tab, xcd_local(blockIdx.x, gridDim.x), loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    ht_tile(m.B, m.Cc, m.Xw, m.Yw, m.nao, m.nd, m.r, q0, m.ldw, loc, lds);
}

__global__ void __launch_bounds__(256, 4) k_b_half_transform64(const BMember *__restrict__ M,
                                                               const int *__restrict__ tab, int c)
{
    __shared__ double lds[TileHalf64::LDS_DOUBLES];
    int loc;
    const BMember &m = M[find_member(tab, xcd_local(blockIdx.x, gridDim.x), loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    ht_tile_tl<TileHalf64>(m.B, m.Cc, m.Xw, m.Yw, m.nao, m.nd, m.r, q0, m.ldw, loc, lds, -1);
}

// Stacked-slab half-transform on the 16 x 16 x 4 engine (the plan's tile 3
// or 4; the schedule keeps members whose chunk of slabs spans 4 GiB or more
// on the 4x4x4 tile).
typedef TileHalf16 TileB16;
__global__ void __launch_bounds__(256, 3) k_b_half_transform16(const BMember *__restrict__ M,
                                                               const int *__restrict__ tab, int c)
{
    extern __shared__ double lds[];
    int loc;
    const BMember &m = M[find_member(tab, xcd_local(blockIdx.x, gridDim.x), loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    ht_tile_flat<TileB16>(m.B, m.Cc, m.Xw, m.Yw, m.nao, m.nd, m.r, q0, nq, m.ldw, loc, lds,
                          m.sym ? m.nd * m.r : -1);
}

// Packed slabs on the 16 x 16 x 4 engine: 128 x 64 tiles per slab.
__global__ void __launch_bounds__(256, 3) k_b_half_transform16_packed(const BMember *__restrict__ M,
                                                                      const int *__restrict__ tab,
                                                                      int c)
{
    extern __shared__ double lds[];
    int loc;
    const BMember &m = M[find_member(tab, xcd_local(blockIdx.x, gridDim.x), loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    ht_tile16_packed<TileB16>(m.B, m.Cc, m.Xw, m.Yw, m.nao, m.nd, m.r, q0, m.ldw, loc, lds,
                              m.sym ? m.nd * m.r : -1);
}

// The exchange on the 16 x 16 x 4 engine (member chunk workspaces are capped
// at 256 MB, so X and Y of a density stay within a buffer resource's reach).
__global__ void __launch_bounds__(256, 3) k_b_exchange(const BMember *__restrict__ M,
                                                       const int *__restrict__ tab, int c)
{
    extern __shared__ double lds[];
    int loc;
    const BMember &m = M[find_member(tab, xcd_local(blockIdx.x, gridDim.x), loc)];
    int q0, nq;
    chunk_of(m, c, q0, nq);
    const int nj = nq * m.r;
    int jlen = cdiv_i(nj, m.nsplit);
    jlen = ((jlen + 15) / 16) * 16;
    ex_tile<TileB16>(m.Xw, m.sym ? m.Xw : m.Yw, m.nsplit > 1 ? m.Kp : m.K, m.nao, m.nd, nj, m.ldw,
                     jlen, c > 0, loc, lds, m.sym);
}

__global__ void __launch_bounds__(256) k_b_mirror(const BMember *__restrict__ M,
                                                  const int *__restrict__ tab)
{
    __shared__ double t[32][33];
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    const int nb = mirror_blocks(m.nao);
    mirror_tile(m.K + (i64)(loc / nb) * m.npos, m.nao, loc % nb, t);
}

__global__ void __launch_bounds__(256) k_b_sum_splits(const BMember *__restrict__ M,
                                                      const int *__restrict__ tab)
{
    int loc;
    const BMember &m = M[find_member(tab, blockIdx.x, loc)];
    sum_tile(m.Kp, m.K, (i64)m.nd * m.npos, m.nsplit, loc);
}

// ------------------------------------------------------------------ launch
static constexpr int kLds16 = (int)sizeof(double) * TileB16::LDS_DOUBLES;

hipError_t prepare_batched_kernels()
{
    hipError_t e = set_dynamic_lds((const void *)k_b_half_transform16, kLds16);
    if (e == hipSuccess)
        e = set_dynamic_lds((const void *)k_b_half_transform16_packed, kLds16);
    if (e == hipSuccess)
        e = set_dynamic_lds((const void *)k_b_exchange, kLds16);
    return e;
}

hipError_t launch_batched_phase(int phase, const BMember *M, const int *tab, int ntiles, int step,
                                hipStream_t s, int arg)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (phase >= kPhaseMSliceC)
        return launch_batched_mixed_phase(phase, M, tab, ntiles, step, s, arg);
    const dim3 g(ntiles);
    switch (phase) {
    case kPhaseMirror: {
        ProfScope ps_("b_mirror", s);
        hipLaunchKernelGGL(k_b_mirror, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhasePack: {
        ProfScope ps_("b_pack", s);
        hipLaunchKernelGGL(k_b_pack, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseDensity: {
        ProfScope ps_("b_density", s);
        hipLaunchKernelGGL(k_b_density, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseProject: {
        ProfScope ps_("b_project", s);
        hipLaunchKernelGGL(k_b_project, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseReduce: {
        ProfScope ps_("b_reduce", s);
        hipLaunchKernelGGL(k_b_reduce, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseCoulomb: {
        ProfScope ps_("b_coulomb", s);
        hipLaunchKernelGGL(k_b_coulomb, g, dim3(256), 0, s, M, tab, (const double *)M);
        break;
    }
    case kPhaseHalf: {
        ProfScope ps_("b_half_transform", s);
        hipLaunchKernelGGL(k_b_half_transform, g, dim3(256), 0, s, M, tab, step);
        break;
    }
    case kPhaseHalf64: {
        ProfScope ps_("b_half_transform", s);
        hipLaunchKernelGGL(k_b_half_transform64, g, dim3(256), 0, s, M, tab, step);
        break;
    }
    case kPhaseHalf16: {
        ProfScope ps_("b_half_transform", s);
        hipLaunchKernelGGL(k_b_half_transform16, g, dim3(TileB16::NTHR), kLds16, s, M, tab, step);
        break;
    }
    case kPhaseHalf16Packed: {
        ProfScope ps_("b_half_transform", s);
        hipLaunchKernelGGL(k_b_half_transform16_packed, g, dim3(TileB16::NTHR), kLds16, s, M, tab,
                           step);
        break;
    }
    case kPhaseFoldUpper: {
        ProfScope ps_("b_fold_upper", s);
        hipLaunchKernelGGL(k_b_fold_upper, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseSymPack: {
        ProfScope ps_("b_sym_pack", s);
        hipLaunchKernelGGL(k_b_sym_pack, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseUnpackJ: {
        ProfScope ps_("b_unpack_j", s);
        hipLaunchKernelGGL(k_b_unpack_j, g, dim3(256), 0, s, M, tab);
        break;
    }
    case kPhaseExchange: {
        ProfScope ps_("b_exchange", s);
        hipLaunchKernelGGL(k_b_exchange, g, dim3(TileB16::NTHR), kLds16, s, M, tab, step);
        break;
    }
    case kPhaseSum: {
        ProfScope ps_("b_sum_splits", s);
        hipLaunchKernelGGL(k_b_sum_splits, g, dim3(256), 0, s, M, tab);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace jk
