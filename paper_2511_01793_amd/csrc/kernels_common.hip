// Size-independent kernels and the dispatch from a run-time probe side to the
// per-side launchers (instantiated in kernels_m32.hip, kernels_m64.hip and
// kernels_m128.hip).
#include "kernels.hpp"

namespace emg {

extern template struct Launchers<32>;
extern template struct Launchers<64>;
extern template struct Launchers<128>;

__global__ __launch_bounds__(256) void k_sum_doubles(const double* in, int count, double* out) {
  __shared__ double redd[16];
  // thread t adds in[t], in[t + 256], ... in that order; eight loads in flight per round
  constexpr int U = 8;
  double acc = 0.0;
  for (int i0 = threadIdx.x; i0 < count; i0 += 256 * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = i0 + 256 * u < count ? in[i0 + 256 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + 256 * u < count) acc += v[u];
  }
  const double tot = block_sum<256>(acc, redd, threadIdx.x);
  if (threadIdx.x == 0) out[0] = tot;
}

__global__ __launch_bounds__(256) void k_zero_doubles(double* p, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

__global__ __launch_bounds__(64) void k_zero_u32(unsigned* p) { p[threadIdx.x] = 0u; }

__global__ __launch_bounds__(256) void k_slot_info(const int* idx, const int2* pos, int n_pos,
                                                   int4* slot, int count) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= count) return;
  const int k = min(max(idx[j], 0), n_pos - 1);
  const int2 p = pos[k];
  slot[j] = make_int4(k, p.x, p.y, 0);
}

__global__ __launch_bounds__(256) void k_fill_c64(float2* p, size_t count, float2 v) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_slot_info(const int* idx, const int2* pos, int n_pos, int4* slot, int count,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_slot_info, dim3((count + 255) / 256), dim3(256), 0, s, idx, pos, n_pos, slot,
                     count);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_zero_doubles(double* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_doubles, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_sum_doubles(const double* in, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(256), 0, s, in, count, out);
  return hipGetLastError();
}

hipError_t launch_fill_c64(float2* p, size_t count, float2 v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_c64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

#define EMG_BY_M(m, CALL)                        \
  switch (m) {                                   \
    case 32: return Launchers<32>::CALL;         \
    case 64: return Launchers<64>::CALL;         \
    case 128: return Launchers<128>::CALL;       \
    case 256: return Launchers256::CALL;         \
    default: return hipErrorInvalidValue;        \
  }

hipError_t launch_patch_step(int m, int v, int L, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
  EMG_BY_M(m, patch_step(v, L, a, s, e0, e1));
}
hipError_t launch_finalize(int m, int f, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  EMG_BY_M(m, finalize(f, a, s, e0, e1));
}
hipError_t launch_patch_step_multi(int m, int v, int L, const StepArgs* args, const int2* work,
                                   int blocks, hipStream_t s) {
  EMG_BY_M(m, patch_step_multi(v, L, args, work, blocks, s));
}
hipError_t launch_finalize_multi(int m, int f, const StepArgs* args, const int2* work, int blocks,
                                 hipStream_t s) {
  EMG_BY_M(m, finalize_multi(f, args, work, blocks, s));
}
hipError_t finalize_item_count(int m, int f, int nr, int nc, int pgroups, int* items) {
  EMG_BY_M(m, finalize_item_count(f, nr, nc, pgroups, items));
}
hipError_t launch_plain_step(int m, int v, int L, const StepArgs& a, hipStream_t s) {
  EMG_BY_M(m, plain_step(v, L, a, s));
}
hipError_t persistent_grid_size(int m, int v, int L, int num_cus, int* grid) {
  EMG_BY_M(m, persistent_grid_size(v, L, num_cus, grid));
}
hipError_t launch_persistent_epoch(int m, int v, int L, const StepArgs& a, int n_pos, int minibatch,
                                   int grid, unsigned* bar, unsigned bar_base, int* err,
                                   unsigned spin_limit, int* used_grid, hipStream_t s) {
  EMG_BY_M(m, persistent_epoch(v, L, a, n_pos, minibatch, grid, bar, bar_base, err, spin_limit,
                               used_grid, s));
}
hipError_t launch_layout_intensities(int m, int v, const float* d, float* dperm, int n_pos,
                                     double* pattern_sums, int* bad_flag, hipStream_t s) {
  EMG_BY_M(m, layout(v, d, dperm, n_pos, pattern_sums, bad_flag, s));
}
hipError_t launch_normalize_probe(int m, float2* probe, double dp_avg, int* zero_flag,
                                  hipStream_t s) {
  EMG_BY_M(m, normalize(probe, dp_avg, zero_flag, s));
}
hipError_t launch_misfit_terms(int m, int v, const float2* obj, int n, const float2* probe,
                               const float* dperm, const int2* pos, const int4* slot, int count,
                               const float2* tw, double* phi_out, int by_pattern, hipStream_t s) {
  EMG_BY_M(m, misfit(v, obj, n, probe, dperm, pos, slot, count, tw, phi_out, by_pattern, s));
}
hipError_t launch_revised_waves(int m, int v, const StepArgs& a, hipStream_t s) {
  EMG_BY_M(m, revised_waves(v, a, s));
}
hipError_t launch_numerators(int m, int v, int L, const StepArgs& a, hipStream_t s) {
  EMG_BY_M(m, numerators(v, L, a, s));
}
hipError_t launch_surrogate_terms(int m, int v, const StepArgs& a, double* terms, hipStream_t s) {
  EMG_BY_M(m, surrogate(v, a, terms, s));
}
hipError_t launch_chain_sweep(int m, int v, int L, const StepArgs& a, int n_steps, hipStream_t s) {
  EMG_BY_M(m, chain(v, L, a, n_steps, s));
}
hipError_t launch_misfit_strips(int m, const StepArgs& a, int k0, int count, double* phi_out,
                                hipStream_t s) {
  if (m != 256) return hipErrorInvalidValue;
  return Launchers256::misfit_strips(a, k0, count, phi_out, s);
}
hipError_t launch_grad(int m, int v, bool f64, const GradArgs& g, hipStream_t s) {
  EMG_BY_M(m, grad(v, f64, g, s));
}

}  // namespace emg
