// gfx950 kernels of the eMAGPIE epoch and their launchers.
//
// One workgroup owns one m x m scan patch in the patch stage: it gathers the
// object window, forms the exit wave psi = Q . z_k (Def. 2.1), runs the
// forward 2-D DFT in LDS, projects onto the measured moduli (Def. 2.1,
// theta(0) = 0), runs the inverse DFT, and applies the per-pixel surrogate
// algebra: the MAGPIE coarse correction (Sec. 3.2, Eqs. 12-15, in its
// block-ratio form), the object numerator conj(Q) R + u z' (Eq. 7 / Eq. 9 as
// a numerator over a denominator), and the probe numerator / denominator of
// Eq. 8.  A finalize stage then sums the numerators over the batch in
// ascending slot order (owner-computes object tiles, fixed-order probe sums),
// divides, and applies the geometric-mean, phase-aligned joint step of Eq. 6.
// No floating-point atomics are used anywhere, so every result is bitwise
// reproducible.
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>

#include "device_fft.hpp"
#include "launch.hpp"

namespace cg = cooperative_groups;

namespace emg {

// ---------------------------------------------------------------------------
// block reductions (wave64 butterflies, then a fixed-order pass over waves)
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void block_max2(float& a, float& b, float* red, int tid) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a = fmaxf(a, __shfl_xor(a, off));
    b = fmaxf(b, __shfl_xor(b, off));
  }
  constexpr int NW = NT / 64;
  if constexpr (NW > 1) {
    const int w = tid >> 6, l = tid & 63;
    if (l == 0) {
      red[w] = a;
      red[NW + w] = b;
    }
    __syncthreads();
    a = red[0];
    b = red[NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
      a = fmaxf(a, red[i]);
      b = fmaxf(b, red[NW + i]);
    }
    __syncthreads();
  }
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red, int tid) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  constexpr int NW = NT / 64;
  if constexpr (NW > 1) {
    const int w = tid >> 6, l = tid & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) v += red[i];
    __syncthreads();
  }
  return v;
}

__device__ __forceinline__ cx<float> ld(const float2* p, size_t i) {
  float2 v = p[i];
  return cx<float>{v.x, v.y};
}
__device__ __forceinline__ void st(float2* p, size_t i, cx<float> v) { p[i] = make_float2(v.re, v.im); }

template <int M>
struct Tile {
  static constexpr int NT = Plan<M>::NT;
  static constexpr int T = NT == 64 ? 16 : (NT == 256 ? 32 : 64);  // object tile side
  static constexpr int PER = T * T / NT;                             // pixels per thread (4)
};

// ---------------------------------------------------------------------------
// per-pixel surrogate algebra for one patch (thread owns a 4 x 4 block)
// ---------------------------------------------------------------------------
template <int M, int L, bool FROM_LDS>
__device__ __forceinline__ void pixel_update(const StepArgs& a, int s, int2 pk, const float2* Rg,
                                             const cx<float>* A, float qqmax, float zmax,
                                             int tid) {
  constexpr int BW = M / 4, LS = lds_stride<M>();
  const int bi = tid / BW, bj = tid % BW;
  const size_t n = (size_t)a.n;
  auto R_at = [&](int r, int c) -> cx<float> {
    if constexpr (FROM_LDS) return A[r * LS + c];
    else return ld(Rg, (size_t)r * M + c);
  };
  // pass 1: 2 x 2 sub-block sums of g = conj(Q)(R - Q z), D, u, Q, |Q|^2
  cx<float> Gs[4], Qs[4];
  float Ds[4], Us[4], Q2s[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    Gs[b] = Qs[b] = cx<float>{0.f, 0.f};
    Ds[b] = Us[b] = Q2s[b] = 0.f;
  }
  if constexpr (L >= 2) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * bi + i, c = 4 * bj + j, sb = (i >> 1) * 2 + (j >> 1);
        const cx<float> q = ld(a.probe, (size_t)r * M + c);
        const cx<float> zz = ld(a.obj, (size_t)(pk.x + r) * n + pk.y + c);
        const cx<float> R = R_at(r, c);
        const float q2 = norm2(q);
        const float u = a.alpha * (qqmax - q2);
        const cx<float> g = cmulc(q, sub(R, mul(q, zz)));
        Gs[sb] = add(Gs[sb], g);
        Ds[sb] += q2 + u;
        Us[sb] += u;
        Qs[sb] = add(Qs[sb], q);
        Q2s[sb] += q2;
      }
    }
  }
  // coarse corrections per 2 x 2 sub-block (block-ratio form of the
  // restricted coarse solve; three levels recurse once more over the 4 x 4)
  cx<float> cc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) cc[b] = cx<float>{0.f, 0.f};
  if constexpr (L == 2) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (Ds[b] > 0.f) cc[b] = scale(Gs[b], 1.f / Ds[b]);
  } else if constexpr (L == 3) {
    cx<float> G2{0.f, 0.f};
    float D2 = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float w = Q2s[b] > 0.f ? norm2(Qs[b]) / (4.f * Q2s[b]) : 0.f;
      G2 = add(G2, scale(Gs[b], w));
      D2 += w * Ds[b];
    }
    const cx<float> c2 = D2 > 0.f ? scale(G2, 1.f / D2) : cx<float>{0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (Ds[b] > 0.f) cc[b] = scale(add(Gs[b], scale(c2, Us[b])), 1.f / Ds[b]);
  }
  // pass 2: numerators and denominators
  const size_t base = (size_t)s * M * M;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * bi + i, c = 4 * bj + j, sb = (i >> 1) * 2 + (j >> 1);
      const cx<float> q = ld(a.probe, (size_t)r * M + c);
      const cx<float> zz = ld(a.obj, (size_t)(pk.x + r) * n + pk.y + c);
      const cx<float> R = R_at(r, c);
      const float q2 = norm2(q);
      const float u = a.alpha * (qqmax - q2);
      const float D = q2 + u;
      const cx<float> zp = add(zz, cc[sb]);
      const cx<float> N = add(cmulc(q, R), scale(zp, u));
      const size_t o = base + (size_t)r * M + c;
      if (a.zplus) {
        st(a.zplus, o, D > 0.f ? scale(N, 1.f / D) : zp);
      } else {
        const float z2 = norm2(zz);
        const float uz = a.alpha_z * (zmax - z2);
        st(a.numer, o, N);
        st(a.pnum, o, add(cmulc(zz, R), scale(q, uz)));
        a.pden[o] = z2 + uz;
        if (s == 0) a.Dbuf[r * M + c] = D;
      }
    }
  }
}

// modulus projection of one thread's 4 x 4 block in transform order:
// Psi' = a Psi/|Psi| (a where Psi = 0), scaled by 1/m^2; returns sum (|Psi| - a)^2
template <int M>
__device__ __forceinline__ double project_block(cx<float>* A, const float* dk, int tid) {
  constexpr int BW = M / 4, LS = lds_stride<M>();
  const int bi = tid / BW, bj = tid % BW;
  const float inv_m2 = 1.f / float(M * M);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * bi + i, c = 4 * bj + j;
      const cx<float> P = A[r * LS + c];
      const float amp = sqrtf(fmaxf(dk[r * M + c], 0.f));
      const float mag = sqrtf(norm2(P));
      const float diff = mag - amp;
      acc += (double)diff * (double)diff;
      const cx<float> o = mag > 0.f ? scale(P, amp / mag) : cx<float>{amp, 0.f};
      A[r * LS + c] = scale(o, inv_m2);
    }
  }
  return acc;
}

// gather psi = Q . z_k into LDS and return max |Q|^2, max |z_k|^2 (all threads)
template <int M>
__device__ __forceinline__ void gather_block(const StepArgs& a, int2 pk, cx<float>* A, float* redf,
                                             float& qqmax, float& zmax, int tid) {
  constexpr int BW = M / 4, LS = lds_stride<M>(), NT = Plan<M>::NT;
  const int bi = tid / BW, bj = tid % BW;
  const size_t n = (size_t)a.n;
  float q2m = 0.f, z2m = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * bi + i, c = 4 * bj + j;
      const cx<float> q = ld(a.probe, (size_t)r * M + c);
      const cx<float> zz = ld(a.obj, (size_t)(pk.x + r) * n + pk.y + c);
      q2m = fmaxf(q2m, norm2(q));
      z2m = fmaxf(z2m, norm2(zz));
      A[r * LS + c] = mul(q, zz);
    }
  }
  block_max2<NT>(q2m, z2m, redf, tid);
  qqmax = q2m;
  zmax = z2m;
  __syncthreads();
}

// the whole patch stage for slot s, LDS-resident
template <int M, int L>
__device__ __forceinline__ void patch_step(const StepArgs& a, int s, cx<float>* A,
                                           const cx<float>* tws, float* redf, double* redd,
                                           int tid) {
  constexpr int NT = Plan<M>::NT;
  const int k = a.idx[s];
  const int2 pk = a.pos[k];
  float qqmax, zmax;
  gather_block<M>(a, pk, A, redf, qqmax, zmax, tid);
  fft2_forward<float, M>(A, tws, tid);
  double acc = project_block<M>(A, a.dperm + (size_t)k * M * M, tid);
  __syncthreads();
  fft2_inverse<float, M>(A, tws, tid);
  pixel_update<M, L, true>(a, s, pk, nullptr, A, qqmax, zmax, tid);
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0 && a.phi) a.phi[s] = tot / (2.0 * M * M);
  __syncthreads();
}

// finalize work item: an object tile (item < ntiles) or NT probe pixels
template <int M>
__device__ __forceinline__ void finalize_item(const StepArgs& a, int item, int ntiles,
                                              const int2* spos, int tid) {
  constexpr int NT = Plan<M>::NT, T = Tile<M>::T, PER = Tile<M>::PER;
  const int n = a.n;
  if (item < ntiles) {
    const int tpr = (n + T - 1) / T;
    const int ty = (item / tpr) * T, tx = (item % tpr) * T;
    cx<float> accn[PER];
    float accd[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      accn[e] = cx<float>{0.f, 0.f};
      accd[e] = 0.f;
    }
    for (int s = 0; s < a.b; ++s) {
      const int2 p = spos[s];
      if (p.x >= ty + T || p.x + M <= ty || p.y >= tx + T || p.y + M <= tx) continue;
      const float2* ns = a.numer + (size_t)s * M * M;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int q = tid + e * NT;
        const int ry = ty + q / T - p.x, rx = tx + q % T - p.y;
        if ((unsigned)ry < (unsigned)M && (unsigned)rx < (unsigned)M) {
          accn[e] = add(accn[e], ld(ns, ry * M + rx));
          accd[e] += a.Dbuf[ry * M + rx];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * NT;
      const int y = ty + q / T, x = tx + q % T;
      if (accd[e] > 0.f && y < n && x < n) {
        const size_t o = (size_t)y * n + x;
        const cx<float> z = ld(a.obj, o);
        st(a.obj, o, aligned_sqrt(z, scale(accn[e], 1.f / accd[e])));
      }
    }
  } else {
    const int r = (item - ntiles) * NT + tid;
    if (a.update_probe && r < M * M) {
      cx<float> mac{0.f, 0.f};
      float eac = 0.f;
      for (int s = 0; s < a.b; ++s) {
        mac = add(mac, ld(a.pnum, (size_t)s * M * M + r));
        eac += a.pden[(size_t)s * M * M + r];
      }
      if (eac > 0.f) {
        const cx<float> q = ld(a.probe, r);
        st(a.probe, r, aligned_sqrt(q, scale(mac, 1.f / eac)));
      }
    }
    if (item == ntiles && tid == 0 && a.sampled) {
      double t = 0.0;
      for (int s = 0; s < a.b; ++s) t += a.phi[s];
      *a.sampled += t;
    }
  }
}

template <int M>
__host__ __device__ inline int finalize_items(int n, int* ntiles_out) {
  constexpr int T = Tile<M>::T, NT = Plan<M>::NT;
  const int tpr = (n + T - 1) / T;
  *ntiles_out = tpr * tpr;
  return tpr * tpr + (M * M + NT - 1) / NT;
}

// ---------------------------------------------------------------------------
// fused path kernels
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void stage_twiddles(const float2* tw, cx<float>* tws, int tid) {
  for (int j = tid; j < M; j += Plan<M>::NT) tws[j] = ld(tw, j);
}

template <int M, int L>
__global__ __launch_bounds__(Plan<M>::NT) void k_patch_step(StepArgs a) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ float redf[32];
  __shared__ double redd[16];
  const int tid = threadIdx.x;
  stage_twiddles<M>(a.tw, tws, tid);
  __syncthreads();
  patch_step<M, L>(a, blockIdx.x, A, tws, redf, redd, tid);
}

template <int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_finalize(StepArgs a, int ntiles) {
  __shared__ int2 spos[kMaxSlots];
  const int tid = threadIdx.x;
  for (int s = tid; s < a.b; s += Plan<M>::NT) spos[s] = a.pos[a.idx[s]];
  __syncthreads();
  finalize_item<M>(a, blockIdx.x, ntiles, spos, tid);
}

// persistent epoch: every minibatch of a sweep in one cooperative launch
template <int M, int L>
__global__ __launch_bounds__(Plan<M>::NT) void k_epoch_persistent(StepArgs a, int n_pos, int B,
                                                                  int ntiles, int nitems) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ float redf[32];
  __shared__ double redd[16];
  __shared__ int2 spos[kMaxSlots];
  constexpr int NT = Plan<M>::NT;
  cg::grid_group grid = cg::this_grid();
  const int tid = threadIdx.x;
  stage_twiddles<M>(a.tw, tws, tid);
  __syncthreads();
  const int* perm = a.idx;
  for (int start = 0; start < n_pos; start += B) {
    StepArgs x = a;
    x.idx = perm + start;
    x.b = min(B, n_pos - start);
    for (int s = blockIdx.x; s < x.b; s += gridDim.x) patch_step<M, L>(x, s, A, tws, redf, redd, tid);
    grid.sync();
    for (int s = tid; s < x.b; s += NT) spos[s] = x.pos[x.idx[s]];
    __syncthreads();
    for (int item = blockIdx.x; item < nitems; item += gridDim.x)
      finalize_item<M>(x, item, ntiles, spos, tid);
    grid.sync();
  }
}

// ---------------------------------------------------------------------------
// plain path: one launch per stage, intermediates in HBM
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_probe_prep(StepArgs a) {
  __shared__ float redf[32];
  const int tid = threadIdx.x;
  float q2m = 0.f, dummy = 0.f;
  for (int r = tid; r < M * M; r += Plan<M>::NT) q2m = fmaxf(q2m, norm2(ld(a.probe, r)));
  block_max2<Plan<M>::NT>(q2m, dummy, redf, tid);
  if (tid == 0) a.qqmax[0] = q2m;
}

template <int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_gather(StepArgs a) {
  __shared__ float redf[32];
  constexpr int BW = M / 4;
  const int tid = threadIdx.x, s = blockIdx.x;
  const int2 pk = a.pos[a.idx[s]];
  const int bi = tid / BW, bj = tid % BW;
  float z2m = 0.f, dummy = 0.f;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * bi + i, c = 4 * bj + j;
      const cx<float> q = ld(a.probe, (size_t)r * M + c);
      const cx<float> zz = ld(a.obj, (size_t)(pk.x + r) * a.n + pk.y + c);
      z2m = fmaxf(z2m, norm2(zz));
      st(a.stack, (size_t)s * M * M + r * M + c, mul(q, zz));
    }
  block_max2<Plan<M>::NT>(z2m, dummy, redf, tid);
  if (tid == 0) a.zmax[s] = z2m;
}

template <int M, bool INV>
__global__ __launch_bounds__(Plan<M>::NT) void k_fft(StepArgs a) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  constexpr int NT = Plan<M>::NT, LS = lds_stride<M>();
  const int tid = threadIdx.x;
  float2* X = a.stack + (size_t)blockIdx.x * M * M;
  stage_twiddles<M>(a.tw, tws, tid);
  for (int e = tid; e < M * M; e += NT) A[(e / M) * LS + e % M] = ld(X, e);
  __syncthreads();
  if (INV) fft2_inverse<float, M>(A, tws, tid);
  else fft2_forward<float, M>(A, tws, tid);
  for (int e = tid; e < M * M; e += NT) st(X, e, A[(e / M) * LS + e % M]);
}

template <int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_project(StepArgs a) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ double redd[16];
  constexpr int NT = Plan<M>::NT, LS = lds_stride<M>();
  const int tid = threadIdx.x, s = blockIdx.x;
  float2* X = a.stack + (size_t)s * M * M;
  for (int e = tid; e < M * M; e += NT) A[(e / M) * LS + e % M] = ld(X, e);
  __syncthreads();
  const double acc = project_block<M>(A, a.dperm + (size_t)a.idx[s] * M * M, tid);
  __syncthreads();
  for (int e = tid; e < M * M; e += NT) st(X, e, A[(e / M) * LS + e % M]);
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0 && a.phi) a.phi[s] = tot / (2.0 * M * M);
}

template <int M, int L>
__global__ __launch_bounds__(Plan<M>::NT) void k_numerators(StepArgs a) {
  const int s = blockIdx.x;
  const int2 pk = a.pos[a.idx[s]];
  pixel_update<M, L, false>(a, s, pk, a.stack + (size_t)s * M * M, nullptr, a.qqmax[0], a.zmax[s],
                            threadIdx.x);
}

// ---------------------------------------------------------------------------
// misfit and gradient
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_misfit(const float2* obj, int n,
                                                        const float2* probe, const float* dperm,
                                                        const int2* pos, const float2* tw,
                                                        double* phi_all) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ float redf[32];
  __shared__ double redd[16];
  constexpr int NT = Plan<M>::NT;
  const int tid = threadIdx.x, k = blockIdx.x;
  stage_twiddles<M>(tw, tws, tid);
  StepArgs a{};
  a.obj = const_cast<float2*>(obj);
  a.n = n;
  a.probe = const_cast<float2*>(probe);
  float qq, zm;
  gather_block<M>(a, pos[k], A, redf, qq, zm, tid);
  fft2_forward<float, M>(A, tws, tid);
  const double acc = project_block<M>(A, dperm + (size_t)k * M * M, tid);
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0) phi_all[k] = tot / (2.0 * M * M);
}

template <typename T>
__device__ __forceinline__ cx<T> ldT(const void* p, size_t i) {
  return reinterpret_cast<const cx<T>*>(p)[i];
}
template <typename T>
__device__ __forceinline__ void stT(void* p, size_t i, cx<T> v) {
  reinterpret_cast<cx<T>*>(p)[i] = v;
}

template <typename T, int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_grad_patch(GradArgs g, int k0) {
  __shared__ cx<T> A[M * lds_stride<M>()];
  __shared__ cx<T> tws[M];
  __shared__ double redd[16];
  constexpr int NT = Plan<M>::NT, BW = M / 4, LS = lds_stride<M>();
  const int tid = threadIdx.x, s = blockIdx.x, k = k0 + s;
  const int bi = tid / BW, bj = tid % BW;
  const int2 pk = g.pos[k];
  const size_t n = (size_t)g.n;
  for (int j = tid; j < M; j += NT) tws[j] = ldT<T>(g.tw, j);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * bi + i, c = 4 * bj + j;
      A[r * LS + c] = mul(ldT<T>(g.probe, (size_t)r * M + c), ldT<T>(g.obj, (pk.x + r) * n + pk.y + c));
    }
  __syncthreads();
  fft2_forward<T, M>(A, tws, tid);
  // residual in Fourier space: Psi - Psi' = (|Psi| - a) Psi/|Psi|, or -a where Psi = 0
  const float* dk = g.dperm + (size_t)k * M * M;
  const T inv_m2 = T(1) / T(M * M);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * bi + i, c = 4 * bj + j;
      const cx<T> P = A[r * LS + c];
      const T amp = sqrt(fmax(T(dk[r * M + c]), T(0)));
      const T mag = sqrt(norm2(P));
      const T diff = mag - amp;
      acc += (double)diff * (double)diff;
      const cx<T> E = mag > T(0) ? scale(P, diff / mag) : cx<T>{-amp, T(0)};
      A[r * LS + c] = scale(E, inv_m2);
    }
  __syncthreads();
  fft2_inverse<T, M>(A, tws, tid);
  const size_t base = (size_t)s * M * M;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * bi + i, c = 4 * bj + j;
      const cx<T> e = A[r * LS + c];
      const cx<T> q = ldT<T>(g.probe, (size_t)r * M + c);
      const cx<T> zz = ldT<T>(g.obj, (pk.x + r) * n + pk.y + c);
      stT<T>(g.gz_slots, base + r * M + c, cmulc(q, e));
      stT<T>(g.gq_slots, base + r * M + c, cmulc(zz, e));
    }
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0) g.phi_all[k] = tot / (2.0 * M * M);
}

template <typename T, int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_grad_scatter(GradArgs g, int k0, int cnt,
                                                              int first) {
  __shared__ int2 spos[kMaxSlots];
  constexpr int NT = Plan<M>::NT, TS = Tile<M>::T, PER = Tile<M>::PER;
  const int tid = threadIdx.x, n = g.n;
  for (int s = tid; s < cnt; s += NT) spos[s] = g.pos[k0 + s];
  __syncthreads();
  const int tpr = (n + TS - 1) / TS;
  const int ty = (blockIdx.x / tpr) * TS, tx = (blockIdx.x % tpr) * TS;
  cx<T> acc[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) acc[e] = cx<T>{T(0), T(0)};
  for (int s = 0; s < cnt; ++s) {
    const int2 p = spos[s];
    if (p.x >= ty + TS || p.x + M <= ty || p.y >= tx + TS || p.y + M <= tx) continue;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * NT;
      const int ry = ty + q / TS - p.x, rx = tx + q % TS - p.y;
      if ((unsigned)ry < (unsigned)M && (unsigned)rx < (unsigned)M)
        acc[e] = add(acc[e], ldT<T>(g.gz_slots, (size_t)s * M * M + ry * M + rx));
    }
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int q = tid + e * NT;
    const int y = ty + q / TS, x = tx + q % TS;
    if (y < n && x < n) {
      const size_t o = (size_t)y * n + x;
      stT<T>(g.gobj, o, first ? acc[e] : add(ldT<T>(g.gobj, o), acc[e]));
    }
  }
}

template <typename T, int M>
__global__ __launch_bounds__(256) void k_grad_probe(GradArgs g, int cnt, int first) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= M * M) return;
  cx<T> acc{T(0), T(0)};
  for (int s = 0; s < cnt; ++s) acc = add(acc, ldT<T>(g.gq_slots, (size_t)s * M * M + r));
  stT<T>(g.gprobe, r, first ? acc : add(ldT<T>(g.gprobe, r), acc));
}

// ---------------------------------------------------------------------------
// init helpers
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_layout(const float* d, float* dperm,
                                                        double* sums, int* bad) {
  __shared__ double redd[16];
  constexpr int NT = Plan<M>::NT;
  const int tid = threadIdx.x, k = blockIdx.x;
  const float* src = d + (size_t)k * M * M;
  float* dst = dperm + (size_t)k * M * M;
  double acc = 0.0;
  int nonfinite = 0;
  for (int e = tid; e < M * M; e += NT) {
    const float v = src[freq_of_pos<M>(e / M) * M + freq_of_pos<M>(e % M)];
    dst[e] = v;
    nonfinite |= !isfinite(v);
    acc += (double)v;
  }
  if (nonfinite) atomicOr(bad, 1);
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0) sums[k] = tot;
}

template <int M>
__global__ __launch_bounds__(Plan<M>::NT) void k_normalize(float2* probe, double dp_avg,
                                                           int* zero_flag) {
  __shared__ double redd[16];
  constexpr int NT = Plan<M>::NT;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int r = tid; r < M * M; r += NT) {
    const float2 v = probe[r];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tot == 0.0) {
    if (tid == 0) zero_flag[0] = 1;
    return;
  }
  const float sc = (float)(dp_avg / sqrt(tot));
  for (int r = tid; r < M * M; r += NT) {
    const float2 v = probe[r];
    probe[r] = make_float2(v.x * sc, v.y * sc);
  }
}

__global__ __launch_bounds__(256) void k_sum_doubles(const double* in, int count, double* out) {
  __shared__ double redd[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) acc += in[i];
  const double tot = block_sum<256>(acc, redd, threadIdx.x);
  if (threadIdx.x == 0) out[0] = tot;
}

__global__ __launch_bounds__(256) void k_zero_doubles(double* p, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define EMG_DISPATCH_M(m, FN, ...)                \
  switch (m) {                                    \
    case 32: return FN<32>(__VA_ARGS__);          \
    case 64: return FN<64>(__VA_ARGS__);          \
    case 128: return FN<128>(__VA_ARGS__);        \
    default: return hipErrorInvalidValue;         \
  }

#define EMG_DISPATCH_ML(m, L, FN, ...)                                          \
  switch (m * 4 + L) {                                                          \
    case 32 * 4 + 1: return FN<32, 1>(__VA_ARGS__);                             \
    case 32 * 4 + 2: return FN<32, 2>(__VA_ARGS__);                             \
    case 32 * 4 + 3: return FN<32, 3>(__VA_ARGS__);                             \
    case 64 * 4 + 1: return FN<64, 1>(__VA_ARGS__);                             \
    case 64 * 4 + 2: return FN<64, 2>(__VA_ARGS__);                             \
    case 64 * 4 + 3: return FN<64, 3>(__VA_ARGS__);                             \
    case 128 * 4 + 1: return FN<128, 1>(__VA_ARGS__);                           \
    case 128 * 4 + 2: return FN<128, 2>(__VA_ARGS__);                           \
    case 128 * 4 + 3: return FN<128, 3>(__VA_ARGS__);                           \
    default: return hipErrorInvalidValue;                                       \
  }

template <int M, int L>
static hipError_t patch_step_l(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_patch_step<M, L>), dim3(a.b), dim3(Plan<M>::NT), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_patch_step(int m, int L, const StepArgs& a, hipStream_t s) {
  EMG_DISPATCH_ML(m, L, patch_step_l, a, s);
}

template <int M>
static hipError_t finalize_l(const StepArgs& a, hipStream_t s) {
  int ntiles;
  const int items = finalize_items<M>(a.n, &ntiles);
  hipLaunchKernelGGL(k_finalize<M>, dim3(items), dim3(Plan<M>::NT), 0, s, a, ntiles);
  return hipGetLastError();
}
hipError_t launch_finalize(int m, const StepArgs& a, hipStream_t s) {
  EMG_DISPATCH_M(m, finalize_l, a, s);
}

template <int M, int L>
static hipError_t plain_step_l(const StepArgs& a, hipStream_t s) {
  constexpr int NT = Plan<M>::NT;
  hipLaunchKernelGGL(k_probe_prep<M>, dim3(1), dim3(NT), 0, s, a);
  hipLaunchKernelGGL(k_gather<M>, dim3(a.b), dim3(NT), 0, s, a);
  hipLaunchKernelGGL((k_fft<M, false>), dim3(a.b), dim3(NT), 0, s, a);
  hipLaunchKernelGGL(k_project<M>, dim3(a.b), dim3(NT), 0, s, a);
  hipLaunchKernelGGL((k_fft<M, true>), dim3(a.b), dim3(NT), 0, s, a);
  hipLaunchKernelGGL((k_numerators<M, L>), dim3(a.b), dim3(NT), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_plain_step(int m, int L, const StepArgs& a, hipStream_t s) {
  EMG_DISPATCH_ML(m, L, plain_step_l, a, s);
}

template <int M, int L>
static hipError_t grid_l(int num_cus, int* grid) {
  int per = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_epoch_persistent<M, L>,
                                                              Plan<M>::NT, 0);
  if (e != hipSuccess) return e;
  *grid = per * num_cus;
  return hipSuccess;
}
hipError_t persistent_grid_size(int m, int L, int num_cus, int* grid) {
  EMG_DISPATCH_ML(m, L, grid_l, num_cus, grid);
}

template <int M, int L>
static hipError_t persistent_l(const StepArgs& a, int n_pos, int B, int grid, hipStream_t s) {
  int ntiles;
  int nitems = finalize_items<M>(a.n, &ntiles);
  StepArgs aa = a;
  void* args[] = {&aa, &n_pos, &B, &ntiles, &nitems};
  const int want = max(min(B, n_pos), nitems);
  const int g = max(1, min(grid, want));
  return hipLaunchCooperativeKernel((const void*)k_epoch_persistent<M, L>, dim3(g),
                                    dim3(Plan<M>::NT), args, 0, s);
}
hipError_t launch_persistent_epoch(int m, int L, const StepArgs& a, int n_pos, int minibatch,
                                   int grid, hipStream_t s) {
  EMG_DISPATCH_ML(m, L, persistent_l, a, n_pos, minibatch, grid, s);
}

hipError_t launch_zero_doubles(double* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_doubles, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_sum_doubles(const double* in, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(256), 0, s, in, count, out);
  return hipGetLastError();
}

template <int M>
static hipError_t layout_l(const float* d, float* dperm, int n_pos, double* sums, int* bad,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_layout<M>, dim3(n_pos), dim3(Plan<M>::NT), 0, s, d, dperm, sums, bad);
  return hipGetLastError();
}
hipError_t launch_layout_intensities(int m, const float* d, float* dperm, int n_pos,
                                     double* pattern_sums, int* bad_flag, hipStream_t s) {
  EMG_DISPATCH_M(m, layout_l, d, dperm, n_pos, pattern_sums, bad_flag, s);
}

template <int M>
static hipError_t normalize_l(float2* probe, double dp_avg, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize<M>, dim3(1), dim3(Plan<M>::NT), 0, s, probe, dp_avg, flag);
  return hipGetLastError();
}
hipError_t launch_normalize_probe(int m, float2* probe, double dp_avg, int* zero_flag,
                                  hipStream_t s) {
  EMG_DISPATCH_M(m, normalize_l, probe, dp_avg, zero_flag, s);
}

template <int M>
static hipError_t misfit_l(const float2* obj, int n, const float2* probe, const float* dperm,
                           const int2* pos, int n_pos, const float2* tw, double* phi_all,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_misfit<M>, dim3(n_pos), dim3(Plan<M>::NT), 0, s, obj, n, probe, dperm, pos,
                     tw, phi_all);
  return hipGetLastError();
}
hipError_t launch_misfit_terms(int m, const float2* obj, int n, const float2* probe,
                               const float* dperm, const int2* pos, int n_pos, const float2* tw,
                               double* phi_all, hipStream_t s) {
  EMG_DISPATCH_M(m, misfit_l, obj, n, probe, dperm, pos, n_pos, tw, phi_all, s);
}

template <typename T, int M>
static hipError_t grad_t(const GradArgs& g, hipStream_t s) {
  constexpr int NT = Plan<M>::NT, TS = Tile<M>::T;
  const int tpr = (g.n + TS - 1) / TS;
  for (int k0 = 0; k0 < g.n_pos; k0 += g.chunk) {
    const int cnt = min(g.chunk, g.n_pos - k0);
    const int first = k0 == 0;
    hipLaunchKernelGGL((k_grad_patch<T, M>), dim3(cnt), dim3(NT), 0, s, g, k0);
    hipLaunchKernelGGL((k_grad_scatter<T, M>), dim3(tpr * tpr), dim3(NT), 0, s, g, k0, cnt, first);
    hipLaunchKernelGGL((k_grad_probe<T, M>), dim3((M * M + 255) / 256), dim3(256), 0, s, g, cnt,
                       first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t launch_grad(int m, bool f64, const GradArgs& g, hipStream_t s) {
  if (f64) {
    switch (m) {
      case 32: return grad_t<double, 32>(g, s);
      case 64: return grad_t<double, 64>(g, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (m) {
    case 32: return grad_t<float, 32>(g, s);
    case 64: return grad_t<float, 64>(g, s);
    case 128: return grad_t<float, 128>(g, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace emg
