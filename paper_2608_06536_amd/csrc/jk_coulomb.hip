// jk_coulomb.hip -- gamma and the Coulomb matrix from the upper triangles of
// full-square symmetric slabs (coulomb_upper.hpp).
#include <type_traits>

#include "coulomb_upper.hpp"
#include "jk_kernels.hpp"

namespace jk {

__global__ void __launch_bounds__(256) k_coulomb_upper(const double *__restrict__ B,
                                                       const double *__restrict__ g,
                                                       double *__restrict__ J, int nao, int naux,
                                                       int nd, double scale, int accumulate)
{
    coulomb_upper_tile(B, g, J, nao, naux, nd, blockIdx.x, scale, accumulate);
}

__global__ void __launch_bounds__(256) k_fold_upper(double *__restrict__ A, int nao)
{
    fold_upper_row(A, nao, blockIdx.x / nao, blockIdx.x % nao);
}

template <int NK>
__global__ void __launch_bounds__(256) k_project_upper(const double *__restrict__ B,
                                                       const double *__restrict__ S,
                                                       double *__restrict__ part, int naux, int nd,
                                                       int nao, int G)
{
    typedef typename std::conditional<NK == 8, TileProject, TileProject16>::type TL;
    __shared__ double lds[TL::LDS_DOUBLES];
    project_upper_tile<TL, NK>(B, S, part, naux, nd, nao, G, blockIdx.x, lds);
}

__global__ void __launch_bounds__(256) k_project_upper_reduce(const double *__restrict__ part,
                                                              double *__restrict__ g, int naux,
                                                              int nd, int npb)
{
    reduce_tile(part, g, naux, nd, npb, blockIdx.x);
}

hipError_t launch_fold_upper(double *A, int nao, int nmat, hipStream_t s)
{
    {
        ProfScope ps_("fold_upper", s);
        hipLaunchKernelGGL(k_fold_upper, dim3(nmat * nao), dim3(256), 0, s, A, nao);
    }
    return hipGetLastError();
}

int project_upper_blocks(int nao, int naux, int nkg, int *G)
{
    *G = pu_group_rows(nao, naux, nkg);
    return pu_pairs(nao, *G);
}

hipError_t launch_project_upper(const double *B, const double *S, double *part, double *g, int nao,
                                int naux, int nd, hipStream_t s, bool sixteen)
{
    if (sixteen && (nd <= 8 || nd > 16))
        return hipErrorInvalidValue;
    const int nqt = cdiv_i(naux, kProjRows), nkg = sixteen ? 1 : cdiv_i(nd, 8);
    int G;
    const int np = project_upper_blocks(nao, naux, nkg, &G);
    {
        ProfScope ps_(sixteen ? "project16" : "project", s);
        if (sixteen)
            hipLaunchKernelGGL(k_project_upper<16>, dim3(np * nqt), dim3(256), 0, s, B, S, part, naux,
                               nd, nao, G);
        else
            hipLaunchKernelGGL(k_project_upper<8>, dim3(np * nqt * nkg), dim3(256), 0, s, B, S, part,
                               naux, nd, nao, G);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    {
        ProfScope ps_("project_reduce", s);
        hipLaunchKernelGGL(k_project_upper_reduce, dim3(reduce_tiles(naux, nd)), dim3(256), 0, s, part,
                           g, naux, nd, np);
    }
    return hipGetLastError();
}

hipError_t launch_coulomb_upper(const double *B, const double *g, double *J, int nao, int naux,
                                int nd, hipStream_t s, double scale, int accumulate)
{
    {
        ProfScope ps_("coulomb", s);
        hipLaunchKernelGGL(k_coulomb_upper, dim3(cu_tiles(nao, nd)), dim3(256), 0, s, B, g, J, nao,
                           naux, nd, scale, accumulate);
    }
    return hipGetLastError();
}

} // namespace jk
