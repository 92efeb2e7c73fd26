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
    // g as an offset in doubles from the start of the workspace (the batch's
    // descriptors): the Coulomb pass reads g through a kernel argument, whose
    // read-only, unaliased loads the compiler makes scalar (one load per
    // wave, not per lane)
    long long goff;
    int nao, naux, nd, r;
    int qc, ldw, nsplit, npb, plen;
    int sym;            // C_L and C_R are one buffer: X only, K on the upper triangle
    // JK_MIXED members: digit planes (single-buffered), their row exponents
    // and strides (slice_core.hpp layout), the FP64 half-transform chunk XY
    int8_t *Bp, *Cp, *XYp;
    int *eB, *eC, *eXY;
    double *XY;
    double *pm;         // the half-transform's partial row maxima of X/Y
    long long bkb, bps, ckb, cps, xkb, xps;
    int mp, kp, cp, cpx;    // padded rows / inner bytes; cpx: [C_L | C_R] rows the products use
    int mpb;                // rows per slab of B's planes (the half-transform's row tiles)
    // Packed-triangular B (jk.h JK_B_PACKED): bslab doubles per slab of B
    // (npos for full squares); gamma pairs B with S = D + D^T folded onto the
    // packed positions, and J is formed packed in D, then written out in full.
    double *S;
    long long bslab;
    int packed;
};

// Table layout: tab[0] = n entries, tab[1 .. n+1] = start offsets (n+1
// values), tab[n+2 .. 2n+2) = member indices.  Returns the member of tile t
// and its tile index within the member.
__device__ __forceinline__ int find_member(const int *__restrict__ tab, int t, int &local)
{
    const int n = tab[0];
    const int *start = tab + 1;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    local = t - start[lo];
    return tab[n + 2 + lo];
}

// Workgroup index remapped so that runs of kXcdRun consecutive table tiles
// (the column tiles of one row panel, the tiles of one exchange row) land on
// one XCD and share its L2, while the table's order (larger tiles first)
// holds at the scale of 8 kXcdRun tiles.  Within each full block of
// 8 kXcdRun indices, logical = block start + (hw % 8) kXcdRun + (hw / 8) %
// kXcdRun (the hardware deals workgroups round-robin over the 8 XCDs); the
// indices of a last, partial block keep their place.
constexpr int kXcdRun = 16;
__device__ __forceinline__ int xcd_local(int hw, int n)
{
    const int blk = 8 * kXcdRun;
    const int b0 = hw - hw % blk;
    if (b0 + blk > n)
        return hw;
    const int r = hw - b0;
    return b0 + (r & 7) * kXcdRun + (r >> 3);
}

// Chunk of member m at step c: first slab and slab count.
__device__ __forceinline__ void chunk_of(const BMember &m, int c, int &q0, int &nq)
{
    q0 = c * m.qc;
    nq = (m.naux - q0) < m.qc ? (m.naux - q0) : m.qc;
}

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
    kPhaseHalf16 = 9,    // the half-transform on the 16 x 16 x 4 engine over stacked slabs
    kPhaseMirror = 10,   // lower triangle of K from the upper (symmetric members)
    kPhaseSymPack = 11,  // packed B: S = D + D^T on the packed positions
    kPhaseUnpackJ = 12,  // packed B: J in full from its packed form
    kPhaseHalf16Packed = 13,  // packed B: the 16 x 16 x 4 half-transform, tiles per slab
    kPhaseFoldUpper = 14,     // full squares: D folded onto its upper triangle (gamma)
    // JK_MIXED phases (jk_mixed.hip)
    kPhaseMSliceC = 20,  // digit planes of [C_L | C_R]
    kPhaseMSliceB = 21,  // digit planes of the chunk's slabs of B
    kPhaseMHalf = 22,    // INT8 half-transform of the chunk
    kPhaseMRowmax = 23,  // row exponents of the chunk's X and Y
    kPhaseMSliceXY = 24, // digit planes of the chunk's X and Y
    kPhaseMExchange = 25, // INT8 exchange of the chunk
    kPhaseMSliceBPacked = 26  // digit planes of the chunk's packed slabs
};

// Sets the dynamic LDS size of the batched kernels that need it on the
// current device (before a launch sequence is captured).
hipError_t prepare_batched_kernels();

// One launch of a phase over the members listed in tab (device pointer):
// ntiles workgroups, step = chunk index for the chunked phases.  arg: the
// slicer's register blocks (kPhaseMSliceB), or 16 x the dynamic LDS bytes
// plus the register blocks (kPhaseMSliceBPacked).
hipError_t launch_batched_phase(int phase, const BMember *M, const int *tab, int ntiles, int step,
                                hipStream_t s, int arg = 0);
hipError_t launch_batched_mixed_phase(int phase, const BMember *M, const int *tab, int ntiles,
                                      int step, hipStream_t s, int arg);
hipError_t prepare_batched_mixed_kernels();

} // namespace jk
