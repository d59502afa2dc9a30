// Peak probes of libpe (pe_probe_peaks): matrix-core throughput with
// register-resident operands and HBM bandwidth of a device copy. Compiled as
// its own unit with MFMA accumulators kept in ordinary vector registers, so
// that the loops hold nothing but the products (the default register
// assignment moves loop-carried FP64 accumulators between register files
// every round).
#include "pe_kernels.h"

namespace pe {

// ---------------------------------------------------------------------------
// peak probes: matrix-core throughput with register-resident operands (ACC
// independent accumulator chains per wave, `iters` rounds) and HBM bandwidth
// of a 16-byte-vector copy
// ---------------------------------------------------------------------------
typedef float pf32x4 __attribute__((ext_vector_type(4)));
typedef double pf64x4 __attribute__((ext_vector_type(4)));
constexpr int PROBE_ACC = 16;

__global__ __launch_bounds__(256) void k_probe_mfma32(int iters, float seed, float* __restrict__ out) {
    pf32x4 acc[PROBE_ACC];
    for (int a = 0; a < PROBE_ACC; ++a) acc[a] = pf32x4{0.f, 0.f, 0.f, 0.f};
    const float x = seed * (float)(threadIdx.x + 1), y = seed * 0.5f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int a = 0; a < PROBE_ACC; ++a) acc[a] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc[a], 0, 0, 0);
    }
    float sum = 0.f;
    for (int a = 0; a < PROBE_ACC; ++a) sum += acc[a][0] + acc[a][1] + acc[a][2] + acc[a][3];
    out[blockIdx.x * (long)blockDim.x + threadIdx.x] = sum;
}

// FP64: 8 chains of two rounds each (16 products per round, as above)
__global__ __launch_bounds__(256) void k_probe_mfma64(int iters, double seed, double* __restrict__ out) {
    constexpr int A64 = PROBE_ACC / 2;
    pf64x4 acc[A64];
    for (int a = 0; a < A64; ++a) acc[a] = pf64x4{0.0, 0.0, 0.0, 0.0};
    const double x = seed * (double)(threadIdx.x + 1), y = seed * 0.5;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int a = 0; a < A64; ++a) acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[a], 0, 0, 0);
    }
    double sum = 0.0;
    for (int a = 0; a < A64; ++a) sum += acc[a][0] + acc[a][1] + acc[a][2] + acc[a][3];
    out[blockIdx.x * (long)blockDim.x + threadIdx.x] = sum;
}

__global__ __launch_bounds__(256) void k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst, long n) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

hipError_t probe_launch(int kind, int blocks, int iters, void* out, const void* src, long n, hipStream_t st) {
    switch (kind) {
        case 0: hipLaunchKernelGGL(k_probe_mfma32, dim3(blocks), dim3(256), 0, st, iters, 1e-3f, (float*)out); break;
        case 1: hipLaunchKernelGGL(k_probe_mfma64, dim3(blocks), dim3(256), 0, st, iters, 1e-3, (double*)out); break;
        default: hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, st, (const float4*)src, (float4*)out, n); break;
    }
    return hipGetLastError();
}

}  // namespace pe
