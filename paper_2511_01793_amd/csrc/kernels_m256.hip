// Probe side m = 256.  A 256 x 256 complex64 tile (512 KiB) exceeds a CU's LDS,
// so one patch runs as 16 row strips and 16 column blocks of 16 lines each, the
// tile passing through the per-minibatch stack buffer (L2/MALL resident) between
// them:
//   1. row strips:    psi = Q . z_k (Def. 2.1), forward row passes, strip maxima
//                     of |Q|^2 and |z_k|^2;
//   2. column blocks: forward column passes, the modulus projection between the
//                     last forward and the first inverse pass (as in the one-
//                     workgroup kernel), inverse column passes, partial misfits;
//   3. row strips:    inverse row passes, then the per-pixel surrogate algebra of
//                     the strip (multigrid blocks of 2 x 2 and 4 x 4 never cross a
//                     strip of 16 rows), numerators for the finalize.
// The radix split is 16 x 16 in both directions, so the transform order (and the
// amplitude layout) is that of the plan (256, 0).  The finalize, layout and
// normalisation kernels are the shared templates.
#include "kernels.hpp"

namespace emg {

namespace big {
constexpr int M = 256, S = 16, NT = 256, LSR = M + 1, LSC = S + 1;
constexpr int R1 = Plan<256, 0>::R1, R2 = Plan<256, 0>::R2;

// thread's 2 x 2 blocks in a 16 x 256 strip: four rounds of 16 x 64 pixels side by
// side; four consecutive lanes own one 4 x 4 region
struct StripLayout {
  static constexpr int ROUNDS = 4;
  __device__ static void origin(int tid, int rd, int& r0, int& c0) {
    const int q = tid >> 2, sub = tid & 3;
    r0 = 4 * (q >> 4) + 2 * (sub >> 1);
    c0 = 4 * (q & 15) + 2 * (sub & 1) + 64 * rd;
  }
};
}  // namespace big

// Every kernel below runs (slot, strip) pairs strip-major: block i takes slot
// i mod b and strip i / b, so with b a multiple of the XCD count all strips of a
// slot run on one XCD (block i runs on XCD i mod 8), beside the slots listed next
// to it, and the overlapping windows' object rows meet in that XCD's L2.
//
// 1. psi and forward row passes of strip rb of slot s (or of pattern k0 + s when
// a.slot is null: the misfit over all patterns)
__global__ __launch_bounds__(256) void k256_rows_fwd(StepArgs a, int k0) {
  using namespace big;
  __shared__ cx<float> A[S * LSR];
  __shared__ cx<float> tws[M];
  __shared__ float redf[2 * NT / 64];
  const int tid = threadIdx.x, nsl = gridDim.x / S, s = blockIdx.x % nsl, rb = blockIdx.x / nsl,
            row0 = rb * S;
  int wr, wc;
  if (a.slot) {
    const int4 sl = a.slot[s];
    wr = sl.y;
    wc = sl.z;
  } else {
    const int2 p = a.pos[k0 + s];
    wr = p.x;
    wc = p.y;
  }
  tws[tid] = ld(a.tw, tid);
  const float2* zwin = a.obj + (size_t)wr * a.n + wc;
  float q2m = 0.f, z2m = 0.f;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    const cx<float> q = ld(a.probe, (size_t)(row0 + r) * M + tid);
    const cx<float> zz = ld(zwin, (size_t)(row0 + r) * a.n + tid);
    q2m = fmaxf(q2m, norm2(q));
    z2m = fmaxf(z2m, norm2(zz));
    A[r * LSR + tid] = mul(q, zz);
  }
  wave_max2_to_lds<NT>(q2m, z2m, redf, tid);
  __syncthreads();
  fft_pass_lines<float, M, R1, R2, S, NT, LSR, false, true, false>(A, tws, tid);
  __syncthreads();
  fft_pass_lines<float, M, R1, R2, S, NT, LSR, false, false, false>(A, tws, tid);
  __syncthreads();
  float qm, zm;
  lds_max2<NT>(redf, qm, zm);
  if (tid == 0) {
    a.part_q[s * S + rb] = qm;
    a.part_z[s * S + rb] = zm;
  }
  // the strip to the stack buffer, written through the L2 (the column blocks read it
  // in the next kernel)
  float2* out = a.stack + (size_t)s * M * M + (size_t)row0 * M;
#pragma unroll
  for (int r = 0; r < S; ++r) st_through(through_buffer(out, S * M), r * M + tid, A[r * LSR + tid]);
}

// 2. column block cb of slot s: forward column passes, then in the pair pass the
// modulus projection (kColsStep), only the misfit terms (kColsMisfit), or the Fourier
// residual of the gradient (kColsGrad: Psi - Psi' = (|Psi| - a) Psi / |Psi|, or -a
// where Psi = 0, scaled by 1/m^2, with the misfit terms of the gradient's own
// arithmetic); inverse column passes (kColsStep, kColsGrad)
constexpr int kColsMisfit = 0, kColsStep = 1, kColsGrad = 2;
template <int MODE>
__global__ __launch_bounds__(256) void k256_cols(StepArgs a, int k0) {
  constexpr bool STEP = MODE == kColsStep, INVERSE = MODE != kColsMisfit;
  using namespace big;
  __shared__ cx<float> A[M * LSC];
  __shared__ cx<float> tws[M];
  __shared__ double redd[NT / 64];
  const int tid = threadIdx.x, nsl = gridDim.x / S, s = blockIdx.x % nsl, cb = blockIdx.x / nsl,
            col0 = cb * S;
  const int k = a.slot ? a.slot[s].x : k0 + s;
  // the pair pass has S * R2 = NT items of R1 points: item tid, line tid % S,
  // positions R1 (tid / S) + j; its amplitudes are loaded first
  const int line = tid % S, g = tid / S;
  const float* dk = a.dperm + (size_t)k * M * M;
  float amp[R1];
#pragma unroll
  for (int j = 0; j < R1; ++j) amp[j] = dk[(size_t)(R1 * g + j) * M + col0 + line];
  tws[tid] = ld(a.tw, tid);
  float2* blk = a.stack + (size_t)s * M * M + col0;
#pragma unroll
  for (int e = 0; e < S; ++e) {
    const int idx = tid + e * NT, row = idx / S, cl = idx % S;
    A[row * LSC + cl] = ld(blk, (size_t)row * M + cl);
  }
  __syncthreads();
  fft_pass_lines<float, M, R1, R2, S, NT, LSC, false, true, true>(A, tws, tid);
  __syncthreads();
  double acc = 0.0;
  float2* ph = (STEP && a.phase) ? a.phase + (size_t)k * M * M : nullptr;
  fft_pass_lines_pair<float, M, R1, R2, S, NT, LSC, true>(A, tid, [&](int e, cx<float>& v) {
    if constexpr (STEP) {
      float2* pe = ph ? ph + (size_t)(R1 * g + e) * M + col0 + line : nullptr;
      acc += (double)project_amp<M>(v, amplitude(amp[e]), pe, a.phase_write != 0);
    } else if constexpr (MODE == kColsGrad) {
      const float am = sqrtf(fmaxf(amp[e], 0.f));
      const float mag = sqrtf(norm2(v));
      const float diff = mag - am;
      acc += (double)diff * (double)diff;
      const cx<float> E = mag > 0.f ? scale(v, diff / mag) : cx<float>{-am, 0.f};
      v = scale(E, 1.f / float(M * M));
    } else {
      cx<float> t = v;
      acc += (double)project_amp<M>(t, amplitude(amp[e]));
    }
  });
  acc = wave_sum(acc);
  if ((tid & 63) == 0) redd[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) a.part_phi[s * S + cb] = lds_sum<NT>(redd);
  if constexpr (INVERSE) {
    fft_pass_lines<float, M, R1, R2, S, NT, LSC, true, true, true>(A, tws, tid);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < S; ++e) {
      const int idx = tid + e * NT, row = idx / S, cl = idx % S;
      st_through(through_buffer(blk, M * M), row * M + cl, A[row * LSC + cl]);
    }
  }
}

// 3. inverse row passes of strip rb of slot s and the strip's per-pixel algebra;
// with STORE_R the revised exit wave R_k of the strip also goes back to the stack
// buffer (the descent check keeps it, frozen, for the surrogate after the step)
template <int L, bool STORE_R = false>
__global__ __launch_bounds__(256) void k256_rows_inv(StepArgs a) {
  using namespace big;
  __shared__ cx<float> A[S * LSR];
  __shared__ cx<float> tws[M];
  const int tid = threadIdx.x, nsl = gridDim.x / S, s = blockIdx.x % nsl, rb = blockIdx.x / nsl,
            row0 = rb * S;
  const int4 sl = a.slot[s];
  tws[tid] = ld(a.tw, tid);
  const float2* in = a.stack + (size_t)s * M * M + (size_t)row0 * M;
#pragma unroll
  for (int r = 0; r < S; ++r) A[r * LSR + tid] = ld(in, (size_t)r * M + tid);
  // max |Q|^2 and max |z_k|^2 over the whole patch, from the strip maxima
  float qqmax = a.part_q[s * S], zmax = a.part_z[s * S];
#pragma unroll
  for (int i = 1; i < S; ++i) {
    qqmax = fmaxf(qqmax, a.part_q[s * S + i]);
    zmax = fmaxf(zmax, a.part_z[s * S + i]);
  }
  if (rb == 0 && tid == 0 && a.phi) {
    double t = a.part_phi[s * S];
    for (int i = 1; i < S; ++i) t += a.part_phi[s * S + i];
    a.phi[s] = t / (2.0 * M * M);
  }
  __syncthreads();
  fft_pass_lines<float, M, R1, R2, S, NT, LSR, true, false, false>(A, tws, tid);
  __syncthreads();
  fft_pass_lines<float, M, R1, R2, S, NT, LSR, true, true, false>(A, tws, tid);
  __syncthreads();
  if constexpr (STORE_R) {
    float2* outR = a.stack + (size_t)s * M * M + (size_t)row0 * M;
#pragma unroll
    for (int r = 0; r < S; ++r) st(outR, (size_t)r * M + tid, A[r * LSR + tid]);
  }
  const size_t n = (size_t)a.n;
  const float2* zwin = a.obj + (size_t)sl.y * n + sl.z;
  pixel_update_ly<M, StripLayout, L, false>(
      a, s, tid, row0,
      [&](int rd, int r0, int c0, cx<float>* q, cx<float>* zz, cx<float>* Rv) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          ld_pair(a.probe, (size_t)(r0 + i) * M + c0, q[2 * i], q[2 * i + 1]);
          zz[2 * i] = ld(zwin, (size_t)(r0 + i) * n + c0);
          zz[2 * i + 1] = ld(zwin, (size_t)(r0 + i) * n + c0 + 1);
          Rv[2 * i] = A[(r0 - row0 + i) * LSR + c0];
          Rv[2 * i + 1] = A[(r0 - row0 + i) * LSR + c0 + 1];
        }
      },
      qqmax, zmax);
}

// per-pattern terms from the 16 partial sums of its column blocks (or strips), in
// block order, times `scale`
__global__ __launch_bounds__(256) void k256_phi_reduce(const double* part_phi, int count,
                                                       double* phi_out, double scale) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  double t = part_phi[i * big::S];
  for (int c = 1; c < big::S; ++c) t += part_phi[i * big::S + c];
  phi_out[i] = t * scale;
}

// gradient: inverse row passes of strip rb of pattern k0 + s turn the Fourier residual
// into e_k = Q z_k - R_k; the strip's slot terms conj(Q) e_k (object) and conj(z_k) e_k
// (probe) go to the gradient slots, for the shared reductions of k_grad_reduce
__global__ __launch_bounds__(256) void k256_rows_grad(StepArgs a, int k0, float2* gz, float2* gq) {
  using namespace big;
  __shared__ cx<float> A[S * LSR];
  __shared__ cx<float> tws[M];
  const int tid = threadIdx.x, nsl = gridDim.x / S, s = blockIdx.x % nsl, rb = blockIdx.x / nsl,
            row0 = rb * S;
  const int2 p = a.pos[k0 + s];
  tws[tid] = ld(a.tw, tid);
  const float2* in = a.stack + (size_t)s * M * M + (size_t)row0 * M;
#pragma unroll
  for (int r = 0; r < S; ++r) A[r * LSR + tid] = ld(in, (size_t)r * M + tid);
  __syncthreads();
  fft_pass_lines<float, M, R1, R2, S, NT, LSR, true, false, false>(A, tws, tid);
  __syncthreads();
  fft_pass_lines<float, M, R1, R2, S, NT, LSR, true, true, false>(A, tws, tid);
  __syncthreads();
  const size_t n = (size_t)a.n, base = (size_t)s * M * M + (size_t)row0 * M;
  const float2* zwin = a.obj + (size_t)(p.x + row0) * n + p.y;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    const cx<float> ev = A[r * LSR + tid];
    const cx<float> q = ld(a.probe, (size_t)(row0 + r) * M + tid);
    const cx<float> zz = ld(zwin, (size_t)r * n + tid);
    st(gz, base + (size_t)r * M + tid, cmulc(q, ev));
    st(gq, base + (size_t)r * M + tid, cmulc(zz, ev));
  }
}

// descent check: 1/2 ||Q . z_k - R_k||^2 (Eq. 3 with R_k frozen in the stack buffer) of
// strip rb of slot s at the current state; FP32 differences, FP64 sum -> part_phi
__global__ __launch_bounds__(256) void k256_surrogate_strips(StepArgs a) {
  using namespace big;
  __shared__ double redd[NT / 64];
  const int tid = threadIdx.x, nsl = gridDim.x / S, s = blockIdx.x % nsl, rb = blockIdx.x / nsl,
            row0 = rb * S;
  const int4 sl = a.slot[s];
  const size_t n = (size_t)a.n;
  const float2* zwin = a.obj + (size_t)(sl.y + row0) * n + sl.z;
  const float2* Rg = a.stack + (size_t)s * M * M + (size_t)row0 * M;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    const cx<float> d = sub(mul(ld(a.probe, (size_t)(row0 + r) * M + tid), ld(zwin, (size_t)r * n + tid)),
                            ld(Rg, (size_t)r * M + tid));
    acc += (double)d.re * (double)d.re + (double)d.im * (double)d.im;
  }
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0) a.part_phi[s * S + rb] = tot;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t Launchers256::patch_step(int v, int L, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                                    hipEvent_t e1) {
  if (v != 0 || L < 1 || L > 3 || !a.part_q || !a.slot) return hipErrorInvalidValue;
  const dim3 grid(a.b * big::S), block(big::NT);
  hipError_t e;
  if (e0 && (e = hipEventRecord(e0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k256_rows_fwd, grid, block, 0, s, a, 0);
  hipLaunchKernelGGL(k256_cols<kColsStep>, grid, block, 0, s, a, 0);
  switch (L) {
    case 1: hipLaunchKernelGGL(k256_rows_inv<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k256_rows_inv<2>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(k256_rows_inv<3>, grid, block, 0, s, a); break;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (e1 && (e = hipEventRecord(e1, s)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t Launchers256::misfit_strips(const StepArgs& a, int k0, int count, double* phi_out,
                                       hipStream_t s) {
  if (!a.part_q || count < 1) return hipErrorInvalidValue;
  StepArgs x = a;
  x.slot = nullptr;
  const dim3 grid(count * big::S), block(big::NT);
  hipLaunchKernelGGL(k256_rows_fwd, grid, block, 0, s, x, k0);
  hipLaunchKernelGGL(k256_cols<kColsMisfit>, grid, block, 0, s, x, k0);
  hipLaunchKernelGGL(k256_phi_reduce, dim3((count + 255) / 256), dim3(256), 0, s,
                     (const double*)x.part_phi, count, phi_out, 1.0 / (2.0 * big::M * big::M));
  return hipGetLastError();
}

hipError_t launch_grad256(const StepArgs& a, const GradArgs& g, hipStream_t s) {
  constexpr int M = 256;
  if (!a.part_q || g.chunk < 1) return hipErrorInvalidValue;
  StepArgs x = a;
  x.slot = nullptr;
  const int tiles = grad_tiles(g), blocks = tiles + grad_probe_blocks(M);
  for (int k0 = 0; k0 < g.n_pos; k0 += g.chunk) {
    const int cnt = min(g.chunk, g.n_pos - k0);
    const dim3 grid(cnt * big::S), block(big::NT);
    hipLaunchKernelGGL(k256_rows_fwd, grid, block, 0, s, x, k0);
    hipLaunchKernelGGL(k256_cols<kColsGrad>, grid, block, 0, s, x, k0);
    hipLaunchKernelGGL(k256_rows_grad, grid, block, 0, s, x, k0, static_cast<float2*>(g.gz_slots),
                       static_cast<float2*>(g.gq_slots));
    hipLaunchKernelGGL(k256_phi_reduce, dim3((cnt + 255) / 256), dim3(256), 0, s,
                       (const double*)x.part_phi, cnt, g.phi_all + k0, 1.0 / (2.0 * M * M));
    const int first = k0 == 0;
    hipLaunchKernelGGL((k_grad_reduce<float, M>), dim3(blocks), dim3(256 * kGradZGroups), 0, s, g,
                       k0, cnt, first, tiles);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_check256(const StepArgs& a, int levels, int finalize_shape, double* out3,
                           hipStream_t s) {
  if (!a.part_q || !a.slot || levels < 1 || levels > 3) return hipErrorInvalidValue;
  const dim3 grid(a.b * big::S), block(big::NT);
  // the step, keeping the revised waves R_k of the state before it in the stack buffer
  hipLaunchKernelGGL(k256_rows_fwd, grid, block, 0, s, a, 0);
  hipLaunchKernelGGL(k256_cols<kColsStep>, grid, block, 0, s, a, 0);
  switch (levels) {
    case 1: hipLaunchKernelGGL((k256_rows_inv<1, true>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k256_rows_inv<2, true>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k256_rows_inv<3, true>), grid, block, 0, s, a); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  StepArgs f = a;
  f.sampled = out3;  // [0] += sum_k Phi_k at the state before the step
  if ((e = Launchers256::finalize(finalize_shape, f, s, nullptr, nullptr)) != hipSuccess) return e;
  // [1] surrogate of Eq. 3 at the new state against the frozen R_k
  hipLaunchKernelGGL(k256_surrogate_strips, grid, block, 0, s, a);
  hipLaunchKernelGGL(k256_phi_reduce, dim3((a.b + 255) / 256), dim3(256), 0, s,
                     (const double*)a.part_phi, a.b, a.phi, 0.5);
  if ((e = launch_sum_doubles(a.phi, a.b, out3 + 1, s)) != hipSuccess) return e;
  // [2] Phi_B at the new state: the batch's misfit terms through the strip kernels
  hipLaunchKernelGGL(k256_rows_fwd, grid, block, 0, s, a, 0);
  hipLaunchKernelGGL(k256_cols<kColsMisfit>, grid, block, 0, s, a, 0);
  hipLaunchKernelGGL(k256_phi_reduce, dim3((a.b + 255) / 256), dim3(256), 0, s,
                     (const double*)a.part_phi, a.b, a.phi, 1.0 / (2.0 * big::M * big::M));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_sum_doubles(a.phi, a.b, out3 + 2, s);
}

hipError_t Launchers256::finalize(int f, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                                  hipEvent_t e1) {
  constexpr int M = 256;
  return with_fin(f, [&](auto fc) {
    constexpr int F = decltype(fc)::value, FNT = FinShape<F>::FNT, T = FinShape<F>::T;
    int ntiles;
    const int items = finalize_items<M, FNT, T>(a.nr, a.n, a.pgroups, &ntiles);
    if (e0) {
      StepArgs aa = a;
      const int4* sl = a.slot;
      float2* ob = a.obj;
      int n = a.n, b = a.b;
      void* args[] = {&sl, &ob, &n, &b, &aa, &ntiles};
      return hipExtLaunchKernel((const void*)k_finalize<M, F>, dim3(items), dim3(FNT), args, 0, s,
                                e0, e1, 0);
    }
    hipLaunchKernelGGL((k_finalize<M, F>), dim3(items), dim3(FNT), 0, s, a.slot, a.obj, a.n, a.b,
                       a, ntiles);
    return hipGetLastError();
  });
}

hipError_t Launchers256::finalize_item_count(int f, int nr, int nc, int pgroups, int* items) {
  return with_fin(f, [&](auto fc) {
    constexpr int F = decltype(fc)::value;
    int ntiles = 0;
    *items = finalize_items<256, FinShape<F>::FNT, FinShape<F>::T>(nr, nc, pgroups, &ntiles);
    return hipSuccess;
  });
}

hipError_t Launchers256::layout(int v, const float* d, float* dperm, int n_pos, double* sums,
                                int* bad, hipStream_t s) {
  if (v != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_layout<256, 0>), dim3(n_pos), dim3(256), 0, s, d, dperm, sums, bad);
  return hipGetLastError();
}

hipError_t Launchers256::normalize(float2* probe, double dp_avg, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize<256>, dim3(1), dim3(256), 0, s, probe, dp_avg, flag);
  return hipGetLastError();
}

hipError_t Launchers256::persistent_grid_size(int, int, int, int* grid) {
  *grid = 0;  // no persistent form at this size
  return hipSuccess;
}

// no m = 256 form (the host rejects these requests before they reach here)
hipError_t Launchers256::patch_step_multi(int, int, const StepArgs*, const int2*, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t Launchers256::finalize_multi(int, const StepArgs*, const int2*, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t Launchers256::plain_step(int, int, const StepArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t Launchers256::persistent_epoch(int, int, const StepArgs&, int, int, int, unsigned*, unsigned,
                                          int*, unsigned, int*, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t Launchers256::misfit(int, const float2*, int, const float2*, const float*, const int2*,
                                const int4*, int, const float2*, double*, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t Launchers256::revised_waves(int, const StepArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t Launchers256::numerators(int, int, const StepArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t Launchers256::surrogate(int, const StepArgs&, double*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t Launchers256::grad(int, bool, const GradArgs&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t Launchers256::chain(int, int, const StepArgs&, int, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace emg
