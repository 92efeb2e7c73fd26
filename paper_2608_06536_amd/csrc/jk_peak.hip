// jk_peak.hip -- matrix-core peak microbenchmark (include/jk_prof.h).
//
// Measures what the device sustains for the two instruction streams of the
// library, so that roofline fractions can be stated against measured as well
// as nominal peaks:
//   INT8  V_MFMA_I32_32X32X32_I8 in the slice engine's pattern: per wave two
//         32 x 32 output tiles, 4 digit fragments of A and 8 of B, the 13
//         digit pairs with i + j <= 6 into 5 level accumulators;
//   FP64  V_MFMA_F64_16X16X4_F64, sixteen independent accumulator chains.
// Operands are per-lane values from a xorshift generator (every byte uniform,
// like the balanced base-256 digits) or constants; the sustained INT8 rate
// depends on the data (the power the matrix cores draw).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/jk_prof.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned xorshift(unsigned &h)
{
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    return h;
}

template <int RANDOM>
__global__ void __launch_bounds__(512) k_peak_i8(int iters, int *__restrict__ sink)
{
    unsigned h = (blockIdx.x * 512u + threadIdx.x) * 2654435761u + 0x9e3779b9u;
    v4i fa[4], fb[2][4];
#pragma unroll
    for (int p = 0; p < 4; p++) {
        fa[p] = RANDOM ? v4i{(int)xorshift(h), (int)xorshift(h), (int)xorshift(h), (int)xorshift(h)}
                       : v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
#pragma unroll
        for (int t = 0; t < 2; t++)
            fb[t][p] = RANDOM ? v4i{(int)xorshift(h), (int)xorshift(h), (int)xorshift(h),
                                    (int)xorshift(h)}
                              : v4i{0x02020202, 0x02020202, 0x02020202, 0x02020202};
    }
    v16i acc[2][5];
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
        for (int l = 0; l < 5; l++)
#pragma unroll
            for (int e = 0; e < 16; e++)
                acc[t][l][e] = 0;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int t = 0; t < 2; t++)
#pragma unroll
                for (int j = 0; j < 4; j++)
                    if (i + j <= 4)
                        acc[t][i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[i], fb[t][j],
                                                                              acc[t][i + j], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
        for (int l = 0; l < 5; l++)
#pragma unroll
            for (int e = 0; e < 16; e++)
                s += acc[t][l][e];
    sink[blockIdx.x * 512 + threadIdx.x] = s;
}

constexpr int kF64Chains = 16;

template <int RANDOM>
__global__ void __launch_bounds__(256, 2) k_peak_f64(int iters, double *__restrict__ sink)
{
    unsigned h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u + 0x7f4a7c15u;
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        a[u] = RANDOM ? (double)xorshift(h) * 0x1p-32 - 0.5 : 0.5;
        b[u] = RANDOM ? (double)xorshift(h) * 0x1p-32 - 0.5 : 0.25;
    }
    v4d acc[kF64Chains];
#pragma unroll
    for (int c = 0; c < kF64Chains; c++)
        acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int c = 0; c < kF64Chains; c++)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c & 3], b[(c >> 2) & 3], acc[c], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kF64Chains; c++)
        s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    sink[blockIdx.x * 256 + threadIdx.x] = s;
}

} // namespace

extern "C" double jk_peak_mfma(int32_t kind, int32_t random)
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
        return -1.0;
    if (kind != 0 && kind != 1)
        return -1.0;
    // four workgroups per CU in sequence (INT8: one 512-thread workgroup fits
    // a CU at a time; FP64: two 256-thread workgroups)
    const int nblk = 4 * ncu;
    const int iters = kind == 0 ? 2000 : 5000;
    void *sink = nullptr;
    if (hipMalloc(&sink, (size_t)nblk * 512 * sizeof(double)) != hipSuccess)
        return -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double rate = -1.0;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        auto launch = [&]() {
            if (kind == 0) {
                if (random)
                    hipLaunchKernelGGL(k_peak_i8<1>, dim3(nblk), dim3(512), 0, 0, iters, (int *)sink);
                else
                    hipLaunchKernelGGL(k_peak_i8<0>, dim3(nblk), dim3(512), 0, 0, iters, (int *)sink);
            } else {
                if (random)
                    hipLaunchKernelGGL(k_peak_f64<1>, dim3(2 * nblk), dim3(256), 0, 0, iters,
                                       (double *)sink);
                else
                    hipLaunchKernelGGL(k_peak_f64<0>, dim3(2 * nblk), dim3(256), 0, 0, iters,
                                       (double *)sink);
            }
        };
        launch();                                  // warm-up (clocks, code load)
        float ms = 0.0f;
        if (hipEventRecord(e0, 0) == hipSuccess) {
            launch();
            if (hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f &&
                hipGetLastError() == hipSuccess) {
                const double ops = kind == 0
                                       ? 2.0 * 32 * 32 * 32 * 26.0 * iters * nblk * 8
                                       : 2.0 * 16 * 16 * 4 * kF64Chains * (double)iters * (2 * nblk) * 4;
                rate = ops / (ms * 1e-3);
            }
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return rate;
}
