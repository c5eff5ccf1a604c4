// The exit-wave misfit of Eq. 1 without a context or a caller workspace, for callers that
// cannot allocate device memory.  Its only scratch (the per-pattern misfit terms) is a
// fixed-size array in the library's own device memory; the twiddles travel in the kernel
// arguments, and the intensities are read in natural order straight from the caller's
// buffer (each one at the position the transform order puts it).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "emagpie.h"
#include "kernels.hpp"

namespace emg {
constexpr int kNoAllocMaxPatterns = 65536;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace emg

// Per-pattern misfit terms of emagpie_misfit_noalloc (512 KiB per device, held until the
// process ends).  Host code never passes this name to a kernel: the device address
// comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[emg::kNoAllocMaxPatterns];

namespace emg {

// failure message for emagpie_last_error (api.hip)
emagpie_status set_error(emagpie_status st, const std::string& msg);

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[kNoAllocMaxDevices] = {};

// the device address of this device's scratch array (looked up at the first call on it)
hipError_t scratch_address(int dev, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

template <int M>
struct Twiddles {
  float2 w[M];  // exp(-2 pi i j / M), evaluated in double on the host, rounded once
};

// window corners clamped into the object, so that every access stays in the buffers
__device__ __forceinline__ int2 clamp_window(int2 p, int nr, int nc, int m) {
  return make_int2(min(max(p.x, 0), nr - m), min(max(p.y, 0), nc - m));
}

template <int M>
__global__ __launch_bounds__((Plan<M, 0>::NT)) void k_misfit_natural(const float2* obj, int nr, int nc,
                                                                   const float2* probe, const float* d,
                                                                   const int2* pos, Twiddles<M> tw,
                                                                   double* terms) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ double redd[16];
  constexpr int NT = Plan<M, 0>::NT;
  const int tid = threadIdx.x, k = blockIdx.x;
  for (int j = tid; j < M; j += NT) tws[j] = cx<float>{tw.w[j].x, tw.w[j].y};
  const int2 pk = clamp_window(pos[k], nr, nc, M);
  const float* dk = d + (size_t)k * M * M;
  const double phi = misfit_pattern<M, 0>(
      obj, nc, probe, pk,
      [&](int r, int c) { return fmaxf(dk[freq_of_pos<M, 0>(r) * M + freq_of_pos<M, 0>(c)], 0.f); },
      A, tws,
      redd, tid);
  if (tid == 0) terms[k] = phi;
}

// m = 128: the two-workgroups-per-CU form of the context's misfit kernel (same
// arithmetic and order of sums, so the two entry points agree bitwise)
template <int M>
__global__ __launch_bounds__(512, 2) void k_misfit_natural_half(const float2* obj, int nr, int nc,
                                                               const float2* probe, const float* d,
                                                               const int2* pos, Twiddles<M> tw,
                                                               double* terms) {
  using HM = HalfMisfit<M, 0>;
  __shared__ cx<float> S[HM::LDS];
  __shared__ cx<float> tws[M];
  __shared__ double redd[16];
  const int tid = threadIdx.x, k = blockIdx.x;
  for (int j = tid; j < M; j += HM::NT) tws[j] = cx<float>{tw.w[j].x, tw.w[j].y};
  __syncthreads();
  const int2 pk = clamp_window(pos[k], nr, nc, M);
  const float* dk = d + (size_t)k * M * M;
  const double phi = misfit_pattern_half<M, 0>(
      obj, nc, probe, pk,
      [&](int r, int c) { return fmaxf(dk[freq_of_pos<M, 0>(r) * M + freq_of_pos<M, 0>(c)], 0.f); },
      S, tws, redd, tid);
  if (tid == 0) terms[k] = phi;
}

template <int M>
hipError_t launch(const float2* obj, int nr, int nc, const float2* probe, const float* d,
                  const int2* pos, int count, double* terms, hipStream_t s) {
  Twiddles<M> tw;
  for (int j = 0; j < M; ++j) {
    const double ang = -2.0 * M_PI * (double)j / (double)M;
    tw.w[j] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  if constexpr (HalfMisfit<M, 0>::value)
    hipLaunchKernelGGL((k_misfit_natural_half<M>), dim3(count), dim3(HalfMisfit<M, 0>::NT), 0, s, obj,
                       nr, nc, probe, d, pos, tw, terms);
  else
    hipLaunchKernelGGL((k_misfit_natural<M>), dim3(count), dim3(Plan<M, 0>::NT), 0, s, obj, nr, nc,
                       probe, d, pos, tw, terms);
  return hipGetLastError();
}

}  // namespace
}  // namespace emg

extern "C" emagpie_status emagpie_misfit_noalloc(int32_t n_rows, int32_t n_cols, int32_t m,
                                                 int32_t n_pos, const int32_t* positions_dev,
                                                 const float* intensities_dev, const void* obj_dev,
                                                 const void* probe_dev, double* misfit_dev,
                                                 void* stream) {
  using emg::set_error;
  if (!positions_dev || !intensities_dev || !obj_dev || !probe_dev || !misfit_dev)
    return set_error(EMAGPIE_E_ARG, "null argument");
  if (m != 32 && m != 64 && m != 128)
    return set_error(m == 256 ? EMAGPIE_E_UNSUPPORTED : EMAGPIE_E_SHAPE,
                     "emagpie_misfit_noalloc takes probe sides 32, 64 and 128");
  if (n_rows < m || n_cols < m || n_rows > 65536 || n_cols > 65536)
    return set_error(EMAGPIE_E_SHAPE, "object sides must satisfy m <= n_rows, n_cols <= 65536");
  if (n_pos < 1 || n_pos > emg::kNoAllocMaxPatterns)
    return set_error(EMAGPIE_E_SHAPE, "emagpie_misfit_noalloc takes 1 to " +
                                          std::to_string(emg::kNoAllocMaxPatterns) + " patterns");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(EMAGPIE_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= emg::kNoAllocMaxDevices) return set_error(EMAGPIE_E_HIP, "device index out of range");
  double* terms = nullptr;
  if ((e = emg::scratch_address(dev, &terms)) != hipSuccess)
    return set_error(EMAGPIE_E_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const auto* o = static_cast<const float2*>(obj_dev);
  const auto* q = static_cast<const float2*>(probe_dev);
  const auto* pos = reinterpret_cast<const int2*>(positions_dev);
  switch (m) {
    case 32: e = emg::launch<32>(o, n_rows, n_cols, q, intensities_dev, pos, n_pos, terms, s); break;
    case 64: e = emg::launch<64>(o, n_rows, n_cols, q, intensities_dev, pos, n_pos, terms, s); break;
    default: e = emg::launch<128>(o, n_rows, n_cols, q, intensities_dev, pos, n_pos, terms, s); break;
  }
  if (e == hipSuccess) e = emg::launch_sum_doubles(terms, n_pos, misfit_dev, s);
  if (e != hipSuccess) return set_error(EMAGPIE_E_HIP, std::string("misfit launch: ") + hipGetErrorString(e));
  return EMAGPIE_OK;
}
