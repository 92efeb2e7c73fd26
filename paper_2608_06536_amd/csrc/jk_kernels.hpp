// jk_kernels.hpp -- launchers of the device kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

typedef int64_t i64;

// Brackets one kernel launch with timing events when jk_prof_enable is on
// (include/jk_prof.h); does nothing otherwise.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    hipStream_t stream_;
    int pair_;
};

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
int exchange_nsplit(int nao, int nd, int nj);
hipError_t launch_exchange(const double *Xw, const double *Yw, double *Kp, int nao, int nd, int nj,
                           int ldw, int nsplit, int accumulate, hipStream_t s);
hipError_t launch_sum_splits(const double *part, double *out, i64 n, int nsplit, hipStream_t s);

// derivative (jk_vjp.hip)
hipError_t launch_omega_expand(const double *om, double *omx, int naux, int nd, int r,
                               hipStream_t s);
hipError_t launch_vjp_stage_b(const double *V, const double *Xw, const double *Yw, double *Pq,
                              double *Rq, int nao, int nd, int r, int nj, int ldw, hipStream_t s);
int vjp_stage_c_nsplit(int nao, int R, int qc);
hipError_t launch_vjp_stage_c(const double *B, const double *Pq, const double *Rq,
                              const double *omx, const double *Cc, double *dCp, int nao, int R,
                              int q0, int nq, int nsplit, int has_v, int has_w, int accumulate,
                              hipStream_t s);
hipError_t launch_vjp_dc_finish(const double *dCp, double *dCL, double *dCR, int nao, int nd,
                                int r, int nsplit, hipStream_t s);
hipError_t launch_vjp_stage_d(const double *Pq, const double *Rq, const double *Cc,
                              const double *omx, const double *gam, const double *W, double *dB,
                              int nao, int nd, int r, int naux, int q0, int nq, int has_v,
                              int has_w, hipStream_t s);

} // namespace jk
