// Calibration kernels for the roofline: a plain device-to-device copy (the
// memory side) and a loop of independent FP32 fused multiply-adds (the vector
// side), built with the same flags as the method's kernels (packed FP32 forms
// disabled, so the FMA rate is that of scalar-lane FP32 operations).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace emg {

// grid-stride copy of n4 16-byte elements: every lane moves 16 B per load and store
__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src,
                                                float4* __restrict__ dst, size_t n4) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

// kChains independent FMA chains per lane, iters rounds; the sum is stored so that
// nothing is dead.  2 * kChains * iters flops per lane.
constexpr int kFmaChains = 16;
__global__ __launch_bounds__(256) void k_fma_loop(float* out, int iters, float a, float b) {
  float v[kFmaChains];
#pragma unroll
  for (int j = 0; j < kFmaChains; ++j) v[j] = 1e-3f * (float)threadIdx.x + (float)j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kFmaChains; ++j) v[j] = __builtin_fmaf(v[j], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kFmaChains; ++j) s += v[j];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

hipError_t launch_copy16(const void* src, void* dst, size_t n4, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(256), 0, s, static_cast<const float4*>(src),
                     static_cast<float4*>(dst), n4);
  return hipGetLastError();
}

hipError_t launch_fma_loop(float* out, int blocks, int iters, hipStream_t s, double* flops) {
  *flops = 2.0 * kFmaChains * (double)iters * 256.0 * (double)blocks;
  hipLaunchKernelGGL(k_fma_loop, dim3(blocks), dim3(256), 0, s, out, iters, 0.999999f, 1e-6f);
  return hipGetLastError();
}

}  // namespace emg
