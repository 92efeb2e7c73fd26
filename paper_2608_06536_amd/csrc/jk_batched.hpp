// jk_batched.hpp -- device descriptor of one member of a batched build.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

// One problem of a batch: its inputs, outputs, the workspace pointers of its
// own single-build plan, and that plan's chunk and split parameters.
struct BMember {
    const double *B, *CL, *CR;
    double *J, *K;
    double *Cc, *D, *part, *g, *Xw, *Yw, *Kp;
    long long npos;
    int nao, naux, nd, r;
    int qc, ldw, nsplit, npb, plen, pad_;
};

enum {
    kPhasePack = 0,
    kPhaseDensity = 1,
    kPhaseProject = 2,
    kPhaseReduce = 3,
    kPhaseCoulomb = 4,
    kPhaseHalf = 5,
    kPhaseExchange = 6,
    kPhaseSum = 7,
    kPhaseHalf64 = 8,    // the half-transform with 64 x 64 tiles (members whose plan chose them)
    kPhaseHalf16 = 9     // the half-transform on the 16 x 16 x 4 engine over stacked slabs
};

// Sets the dynamic LDS size of the batched kernels that need it on the
// current device (before a launch sequence is captured).
hipError_t prepare_batched_kernels();

// One launch of a phase over the members listed in tab (device pointer):
// ntiles workgroups, step = chunk index for the chunked phases.
hipError_t launch_batched_phase(int phase, const BMember *M, const int *tab, int ntiles, int step,
                                hipStream_t s);

} // namespace jk
