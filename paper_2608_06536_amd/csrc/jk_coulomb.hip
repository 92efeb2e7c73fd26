// jk_coulomb.hip -- the Coulomb matrix from the upper triangle of full-square
// slabs (coulomb_upper.hpp).
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
