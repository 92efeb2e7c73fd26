// jk_kernels.hpp -- launchers of the device kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

typedef int64_t i64;

hipError_t launch_pack_c(const double *CL, const double *CR, double *Cc, int nao, int nd, int r,
                         hipStream_t s);
hipError_t launch_density(const double *CL, const double *CR, double *D, int nao, int nd, int r,
                          hipStream_t s);
int project_nblocks(int64_t npos, int naux, int nd, int *plen);
hipError_t launch_project(const double *B, const double *A, double *part, double *g, int naux,
                          int nd, int64_t npos, hipStream_t s);
hipError_t launch_coulomb(const double *B, const double *g, double *J, int naux, int nd,
                          int64_t npos, hipStream_t s);
hipError_t launch_half_transform(const double *B, const double *Cc, double *Xw, double *Yw,
                                 int nao, int nd, int r, int q0, int nq, int ldw, hipStream_t s);
hipError_t launch_exchange(const double *Xw, const double *Yw, double *K, int nao, int nd, int nj,
                           int ldw, int accumulate, hipStream_t s);

} // namespace jk
