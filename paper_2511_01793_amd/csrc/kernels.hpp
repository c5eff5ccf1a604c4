// gfx950 kernels of the eMAGPIE epoch and their launchers, templated on the
// probe side M, the FFT plan variant V, the multigrid depth L and the finalize
// shape F (plans.hpp).  Each probe side is instantiated in a translation unit
// of its own (kernels_m32.hip, kernels_m64.hip, kernels_m128.hip).
//
// One workgroup owns one m x m scan patch in the patch stage: it gathers the
// object window, forms the exit wave psi = Q . z_k (Def. 2.1), runs the
// forward 2-D DFT (LDS passes; one m = 64 plan keeps each line in registers
// across lanes instead, and one m = 128 plan gathers straight into the registers
// of its first pass), projects onto the measured moduli (Def. 2.1,
// theta(0) = 0), runs the inverse DFT, and applies the per-pixel surrogate
// algebra: the MAGPIE coarse correction (Sec. 3.2, Eqs. 12-15, in its
// block-ratio form), the object numerator conj(Q) R + u z' (Eq. 7 / Eq. 9 as
// a numerator over a denominator), and the probe numerator / denominator of
// Eq. 8.  A finalize stage then sums the numerators over the batch in
// ascending slot order (owner-computes object tiles, fixed-shape probe sums),
// divides, and applies the geometric-mean, phase-aligned joint step of Eq. 6.
// No floating-point atomics are used anywhere, so every result is bitwise
// reproducible, and every launch strategy runs the same arithmetic.
//
// The chain of minibatches is sequential (each one reads the state the
// previous one wrote), so at the benchmark's sizes the patch stage is bound by
// latency, not bandwidth: a patch gets up to 1024 threads (16 waves) and each
// thread issues its probe, object and amplitude loads before any dependent work.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_fft.hpp"
#include "launch.hpp"

namespace emg {

// ---------------------------------------------------------------------------
// reductions.  Within a wave: DPP lane permutes (quad swaps, then the half-row
// and row mirrors) leave every lane of a 16-lane row with its row's total; the
// four row totals are combined in a fixed order through readlane.  Across the
// waves of a block: one value per wave in LDS, combined in wave order.  All
// orders are fixed, so every sum is bitwise reproducible.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E, kDppRowHalfMirror = 0x141,
              kDppRowMirror = 0x140;

__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp_f<kDppQuadXor1>(v));
  v = fmaxf(v, dpp_f<kDppQuadXor2>(v));
  v = fmaxf(v, dpp_f<kDppRowHalfMirror>(v));
  v = fmaxf(v, dpp_f<kDppRowMirror>(v));
  return fmaxf(fmaxf(lane_f(v, 0), lane_f(v, 16)), fmaxf(lane_f(v, 32), lane_f(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppQuadXor1>(v);
  v += dpp_d<kDppQuadXor2>(v);
  v += dpp_d<kDppRowHalfMirror>(v);
  v += dpp_d<kDppRowMirror>(v);
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// wave partials to LDS (one lane per wave); the caller orders them with a barrier
template <int NT>
__device__ __forceinline__ void wave_max2_to_lds(float a, float b, float* red, int tid) {
  a = wave_max(a);
  b = wave_max(b);
  if ((tid & 63) == 0) {
    red[tid >> 6] = a;
    red[NT / 64 + (tid >> 6)] = b;
  }
}
template <int NT>
__device__ __forceinline__ void lds_max2(const float* red, float& a, float& b) {
  a = red[0];
  b = red[NT / 64];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {
    a = fmaxf(a, red[i]);
    b = fmaxf(b, red[NT / 64 + i]);
  }
}
template <int NT>
__device__ __forceinline__ double lds_sum(const double* red) {
  double v = red[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) v += red[i];
  return v;
}

template <int NT>
__device__ __forceinline__ void block_max2(float& a, float& b, float* red, int tid) {
  wave_max2_to_lds<NT>(a, b, red, tid);
  __syncthreads();
  lds_max2<NT>(red, a, b);
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red, int tid) {
  v = wave_sum(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  v = lds_sum<NT>(red);
  __syncthreads();
  return v;
}

// sum over the four consecutive lanes of a 4 x 4 region (identical in all four)
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp_f<kDppQuadXor1>(v);
  return v + dpp_f<kDppQuadXor2>(v);
}

__device__ __forceinline__ cx<float> ld(const float2* p, size_t i) {
  float2 v = p[i];
  return cx<float>{v.x, v.y};
}
// 32-bit element offset: the load takes the base in scalar registers
__device__ __forceinline__ cx<float> ld32(const float2* p, unsigned i) {
  float2 v = p[i];
  return cx<float>{v.x, v.y};
}
__device__ __forceinline__ void st(float2* p, size_t i, cx<float> v) { p[i] = make_float2(v.re, v.im); }
// two consecutive complex values at an even index of a 16-byte aligned array
__device__ __forceinline__ void ld_pair(const float2* p, size_t i, cx<float>& a, cx<float>& b) {
  const float4 v = *reinterpret_cast<const float4*>(p + i);
  a = cx<float>{v.x, v.y};
  b = cx<float>{v.z, v.w};
}
__device__ __forceinline__ void st_pair(float2* p, size_t i, cx<float> a, cx<float> b) {
  *reinterpret_cast<float4*>(p + i) = make_float4(a.re, a.im, b.re, b.im);
}

// Stores that write through this XCD's L2 (the agent-scope cache policy).  The
// per-slot numerators are read back by the finalize, a later kernel spread over every
// XCD; held dirty in the writer's L2 they would only be written back at the kernel
// boundary, after the last workgroup, instead of beside the arithmetic.  The m = 256
// stages write the per-minibatch stack buffer the same way.  A raw buffer over one
// slot's values (byte offsets below 2^31).
constexpr int kBufferWord3 = 0x00020000;  // raw buffer of dwords (gfx9 resource word 3)
constexpr int kCachePolicyThrough = 16;   // sc1: coherent at agent scope
__device__ __forceinline__ __amdgpu_buffer_rsrc_t through_buffer(float2* base, int m2) {
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, m2 * (int)sizeof(float2), kBufferWord3);
}
__device__ __forceinline__ void st_through(__amdgpu_buffer_rsrc_t r, int i, cx<float> a) {
  typedef int v2i __attribute__((ext_vector_type(2)));
  const v2i v = {__float_as_int(a.re), __float_as_int(a.im)};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, i * (int)sizeof(float2), 0, kCachePolicyThrough);
}
__device__ __forceinline__ void st_pair_through(__amdgpu_buffer_rsrc_t r, int i, cx<float> a,
                                                cx<float> b) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  const v4i v = {__float_as_int(a.re), __float_as_int(a.im), __float_as_int(b.re),
                 __float_as_int(b.im)};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, i * (int)sizeof(float2), 0, kCachePolicyThrough);
}


template <int M, int V>
struct Px {
  static constexpr int NT = Plan<M, V>::NT, LS = lds_stride<M>();
  // every thread owns 2 x 2 pixel blocks: one per round, ROUNDS rounds
  static constexpr int ROUNDS = M * M / (4 * NT);
  static constexpr int PX = 4 * ROUNDS;  // pixels per thread
  // a round covers RH x RW pixels (RW = min(M, 64) columns); RPC rounds sit
  // side by side, and the round rows stack downwards
  static constexpr int RW = M < 64 ? M : 64;
  static constexpr int RH = 4 * NT / RW;
  static constexpr int RPC = M / RW;
  static constexpr int QW = RW / 4;  // 4 x 4 regions per row of a round
  // one round: keep the thread's probe / object values in registers from the
  // gather to the numerators; several rounds reload them (register budget)
  static constexpr bool CACHE = ROUNDS == 1;
  static_assert(ROUNDS * 4 * NT == M * M && RH % 4 == 0 && RH * (ROUNDS / RPC) == M, "round tiling");
};

// Top-left pixel (r0, c0) of the thread's 2 x 2 block in round rd (c0 is even).
template <int M, int V>
__device__ __forceinline__ void blk_origin(int tid, int rd, int& r0, int& c0) {
  using P = Px<M, V>;
  const int q = tid >> 2, sub = tid & 3;
  r0 = 4 * (q / P::QW) + 2 * (sub >> 1);
  c0 = 4 * (q % P::QW) + 2 * (sub & 1);
  if constexpr (P::ROUNDS > 1) {
    r0 += P::RH * (rd / P::RPC);
    c0 += P::RW * (rd % P::RPC);
  }
}

// Pixel e of a thread: round e / 4, position (e / 2 % 2, e % 2) inside that
// round's 2 x 2 block.  Four consecutive lanes own the four 2 x 2 blocks of one
// 4 x 4 region, so a region-wide sum is two quad lane exchanges.
template <int M, int V>
__device__ __forceinline__ void pix_rc(int tid, int e, int& r, int& c) {
  using P = Px<M, V>;
  const int q = tid >> 2, sub = tid & 3, round = e >> 2;
  r = 4 * (q / P::QW) + 2 * (sub >> 1) + ((e >> 1) & 1);
  c = 4 * (q % P::QW) + 2 * (sub & 1) + (e & 1);
  if constexpr (P::ROUNDS > 1) {
    r += P::RH * (round / P::RPC);
    c += P::RW * (round % P::RPC);
  }
}

// ---------------------------------------------------------------------------
// per-pixel surrogate algebra for one patch, one 2 x 2 block (round) at a time
//   load(rd, r0, c0, q, z, R) fills the probe, object window and revised exit
//   wave of the block at (r0, c0); element 2 i + j is pixel (r0 + i, c0 + j)
// ---------------------------------------------------------------------------
// DIRECT (minibatch of one slot, the whole step in one workgroup): instead of
// storing numerators for the finalize, apply the finalize's arithmetic here --
// sums that start from zero, z+ = N / D and Q+ = M / E, the joint step -- and write
// the object window and the probe in place.  Every pixel has one owner thread.
// LY gives the thread's 2 x 2 blocks: LY::ROUNDS and LY::origin(tid, rd, r0, c0) in
// patch coordinates, to which row0 is added (a strip of a larger patch).
template <int M, int V>
struct PxLayout {
  static constexpr int ROUNDS = Px<M, V>::ROUNDS;
  __device__ static void origin(int tid, int rd, int& r0, int& c0) { blk_origin<M, V>(tid, rd, r0, c0); }
};

// Quotients of the step (the coarse correction's, z+ = N / D and Q+ = M / E) use the
// hardware reciprocal (within one ulp, one instruction) instead of a correctly rounded
// division (about ten).  A last-bit difference in a quotient is far below the step's
// own FP32 rounding.  A divisor below the smallest normal float counts as zero (no
// correction, the pixel left as it was), so the approximation never sees a subnormal
// input.  Every path applies the same arithmetic, so they stay bitwise identical.
constexpr float kMinDivisor = 1.17549435e-38f;  // FLT_MIN
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ZP: the launch writes MAGPIE's z+ (a.zplus) instead of the numerators
template <int M, class LY, int L, bool DIRECT, bool ZP, class LOAD>
__device__ __forceinline__ void pixel_update_body(const StepArgs& a, int s, int tid, int row0,
                                                  LOAD& load, float qqmax, float zmax) {
  const size_t base = (size_t)s * M * M;
  const bool slot_den = a.pden_slot != nullptr;
#pragma unroll
  for (int rd = 0; rd < LY::ROUNDS; ++rd) {
    int r0, c0;
    LY::origin(tid, rd, r0, c0);
    r0 += row0;
    cx<float> q[4], zz[4], R[4];
    load(rd, r0, c0, q, zz, R);
    // per pixel: |Q|^2, u, D = |Q|^2 + u, conj(Q) R (shared by the coarse-grid residual
    // g = conj(Q)(R - Q z) = conj(Q) R - |Q|^2 z and the object numerator)
    float q2[4], u[4], D[4];
    cx<float> cqR[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      q2[e] = norm2(q[e]);
      u[e] = a.alpha * (qqmax - q2[e]);
      D[e] = q2[e] + u[e];
      cqR[e] = cmulc(q[e], R[e]);
    }
    // block sums of g, D, u, Q, |Q|^2
    cx<float> Gs{0.f, 0.f}, Qs{0.f, 0.f};
    float Ds = 0.f, Us = 0.f, Q2s = 0.f;
    if constexpr (L >= 2) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        Gs = add(Gs, axpy(-q2[e], zz[e], cqR[e]));
        Ds += D[e];
        Us += u[e];
        Qs = add(Qs, q[e]);
        Q2s += q2[e];
      }
    }
    // coarse correction of this 2 x 2 block: block-ratio form of the restricted
    // coarse solve; three levels recurse once more over the 4 x 4 region
    cx<float> cc{0.f, 0.f};
    if constexpr (L == 2) {
      if (Ds >= kMinDivisor) cc = scale(Gs, hw_rcp(Ds));
    } else if constexpr (L == 3) {
      const float w = Q2s >= kMinDivisor ? norm2(Qs) * hw_rcp(4.f * Q2s) : 0.f;
      const cx<float> G2{quad_sum(w * Gs.re), quad_sum(w * Gs.im)};
      const float D2 = quad_sum(w * Ds);
      const cx<float> c2 = D2 >= kMinDivisor ? scale(G2, hw_rcp(D2)) : cx<float>{0.f, 0.f};
      if (Ds >= kMinDivisor) cc = scale(axpy(Us, c2, Gs), hw_rcp(Ds));
    }
    // numerators N = conj(Q) R + u z', M = conj(z) R + u_z Q and denominators
    cx<float> N[4], Mn[4];
    float E[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const cx<float> zp = add(zz[e], cc);
      N[e] = axpy(u[e], zp, cqR[e]);
      if constexpr (ZP) {
        N[e] = D[e] >= kMinDivisor ? scale(N[e], hw_rcp(D[e])) : zp;
      } else {
        const float z2 = norm2(zz[e]);
        const float uz = a.alpha_z * (zmax - z2);
        Mn[e] = axpy(uz, q[e], cmulc(zz[e], R[e]));
        E[e] = z2 + uz;
      }
    }
    if constexpr (DIRECT) {
      const int4 sl = a.slot[s];
      const cx<float> zero{0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + (e >> 1), c = c0 + (e & 1);
        const float dd = 0.f + D[e];
        if (dd >= kMinDivisor) {
          const cx<float> zp = scale(add(zero, N[e]), hw_rcp(dd));
          st(a.obj, (size_t)(sl.y + r) * a.n + sl.z + c, a.joint ? aligned_sqrt(zz[e], zp) : zp);
        }
        if (a.update_probe) {
          const float et = 0.f + (slot_den ? zmax : E[e]);
          if (et >= kMinDivisor) {
            const cx<float> qp = scale(add(zero, Mn[e]), hw_rcp(et));
            st(a.probe, (size_t)r * M + c, a.joint ? aligned_sqrt(q[e], qp) : qp);
          }
        }
      }
      continue;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const size_t o = base + (size_t)(r0 + i) * M + c0;
      if constexpr (ZP) {
        st_pair(a.zplus, o, N[2 * i], N[2 * i + 1]);
      } else {
        // the slot's numerator buffers, written through the L2
        const int ob = (r0 + i) * M + c0;  // o - base
        st_pair_through(through_buffer(a.numer + base, M * M), ob, N[2 * i], N[2 * i + 1]);
        st_pair_through(through_buffer(a.pnum + base, M * M), ob, Mn[2 * i], Mn[2 * i + 1]);
        if (!slot_den)
          *reinterpret_cast<float2*>(a.pden + o) = make_float2(E[2 * i], E[2 * i + 1]);
        if (s == 0)
          *reinterpret_cast<float2*>(a.Dbuf + (r0 + i) * M + c0) = make_float2(D[2 * i], D[2 * i + 1]);
      }
    }
  }
  // alpha_z = 1: the probe denominator |z_k|^2 + u_z = max |z_k|^2 is one number per patch
  if (!DIRECT && !ZP && slot_den && tid == 0) a.pden_slot[s] = zmax;
}

// The z+ output is a uniform choice: each case has a copy of the loop, so neither
// tests it per pixel (the minibatch-1 update of DIRECT never writes z+).
template <int M, class LY, int L, bool DIRECT, class LOAD>
__device__ __forceinline__ void pixel_update_ly(const StepArgs& a, int s, int tid, int row0,
                                                LOAD load, float qqmax, float zmax) {
  if (!DIRECT && a.zplus)
    pixel_update_body<M, LY, L, false, true>(a, s, tid, row0, load, qqmax, zmax);
  else
    pixel_update_body<M, LY, L, DIRECT, false>(a, s, tid, row0, load, qqmax, zmax);
}

template <int M, int V, int L, bool DIRECT = false, class LOAD>
__device__ __forceinline__ void pixel_update(const StepArgs& a, int s, int tid, LOAD load,
                                             float qqmax, float zmax) {
  pixel_update_ly<M, PxLayout<M, V>, L, DIRECT, LOAD>(a, s, tid, 0, load, qqmax, zmax);
}

// modulus projection of one pixel in transform order: Psi' = a Psi/|Psi|
// (a where Psi = 0), scaled by 1/m^2; returns (|Psi| - a)^2.  The unit phase
// factor Psi/|Psi| uses the hardware reciprocal square root (within one ulp)
// instead of a correctly rounded square root and division.  |Psi|^2 below the
// smallest normal float (|Psi| < 1.1e-19) counts as zero: theta := 0 there.
// Written with selects only, so no lane branches.
//
// With a phase memory ph (the stateful rule stated after Eq. 3), a zero bin takes
// the unit phasor stored at the pattern's previous visit instead of theta = 0, and
// a live bin stores its phasor Psi/|Psi| when `write` is set.  The memory starts
// at (1, 0), which reproduces theta = 0 at the first visit.
template <int M>
__device__ __forceinline__ float project_amp(cx<float>& P, float amp, float2* ph = nullptr,
                                             bool write = false) {
  constexpr float kTiny = 1.17549435e-38f;  // FLT_MIN
  constexpr float kInvM2 = 1.f / float(M * M);
  const float p2 = norm2(P);
  const bool live = p2 >= kTiny;
  const float ir = __builtin_amdgcn_rsqf(fmaxf(p2, kTiny));
  const float diff = (live ? p2 * ir : 0.f) - amp;
  const float f = amp * ir * kInvM2;
  if (ph) {
    if (live) {
      if (write) *ph = make_float2(P.re * ir, P.im * ir);
      P = cx<float>{P.re * f, P.im * f};
    } else {
      const float2 u = *ph;
      const float s = amp * kInvM2;
      P = cx<float>{s * u.x, s * u.y};
    }
  } else {
    P.re = live ? P.re * f : amp * kInvM2;
    P.im = live ? P.im * f : 0.f;
  }
  return diff * diff;
}
// measured amplitude a = sqrt(max(d, 0)) of one laid-out intensity (hardware square
// root, within one ulp): the layout (k_layout) stores max(d, 0), so d >= 0 here
__device__ __forceinline__ float amplitude(float d) { return __builtin_amdgcn_sqrtf(d); }
template <int M>
__device__ __forceinline__ float project_px(cx<float>& P, float dval, float2* ph = nullptr,
                                            bool write = false) {
  return project_amp<M>(P, amplitude(dval), ph, write);
}

// ---------------------------------------------------------------------------
// pieces of the register-pass plan (m = 64, 8 * 8 split, 1024 threads).  Waves
// 0..7 transform: wave w holds rows 8 w .. 8 w + 7 in the row phase and columns
// 8 w .. 8 w + 7 in the column phase, lane lo + 8 gi taking line lo of the
// wave, 8 points per lane; the tile sits in LDS at xl_addr.  Waves 8..15 stage
// the pattern's amplitudes in LDS (row stride m + 1) meanwhile.
// ---------------------------------------------------------------------------
// twiddles W^(gi j), j = 1..7, of lane group gi: the same in every strided pass
__device__ __forceinline__ void xl_twiddles(const cx<float>* tws, int gi, cx<float>* w) {
#pragma unroll
  for (int j = 1; j < 8; ++j) w[j] = tws[gi * j];
}

// forward row passes of row r: natural order in, row-transform order out
__device__ __forceinline__ void xl_rows_forward(cx<float>* A, const cx<float>* w, int r, int gi) {
  cx<float> v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = A[xl_addr(r, gi + 8 * j)];
  xl_strided<false>(v, w);
  xl_transpose8(v);
  dft8<float, false>(v);
#pragma unroll
  for (int j = 0; j < 8; ++j) A[xl_addr(r, 8 * gi + j)] = v[j];
}

// forward column passes of column C: v[j] is then the spectrum at transform-order
// row 8 gi + j
__device__ __forceinline__ void xl_cols_forward(const cx<float>* A, const cx<float>* w, int C,
                                                int gi, cx<float>* v) {
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = A[xl_addr(gi + 8 * j, C)];
  xl_strided<false>(v, w);
  xl_transpose8(v);
  dft8<float, false>(v);
}

// waves 8..15: the amplitudes sqrt(max(d, 0)) of dk (transform order) to LDS;
// ampv holds the thread's eight intensities (element (tid - 512) + 512 j)
template <int M>
__device__ __forceinline__ void xl_stage_amps(float* ampl, const float* ampv, int tid) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = (tid - 512) + 512 * j;
    ampl[(e / M) * (M + 1) + e % M] = amplitude(ampv[j]);
  }
}

// ---------------------------------------------------------------------------
// the whole patch stage for slot s, LDS-resident
// ---------------------------------------------------------------------------
// Returns the slot's sampled misfit (in thread 0).
// STAGE: the twiddle table is loaded here (its load goes out beside the slot's,
// its LDS copy is written before the first barrier) instead of by the caller.
//
// Plans with register-resident passes (XL; m = 64, 8 * 8 split, 1024 threads):
// the loads, the exit waves and the per-pixel phase are the LDS plan's, the
// tile in LDS in the swizzled layout of xl_addr.  Waves 0..7 transform it, wave
// w holding rows 8 w .. 8 w + 7 in the row phase and columns 8 w .. 8 w + 7 in
// the column phase (a line in 8 lanes, 8 points per lane), so the tile goes
// through LDS between the row and the column phases, not between the two passes
// of a dimension; waves 8..15 meanwhile
// put the pattern's amplitudes in LDS in the column phase's order.  The sampled
// misfit sums the same per-pixel terms as the LDS plans, in another order.
//
// PH = false: the context keeps no phase memory (a.phase is null), and the
// projection is compiled without it; PH = true tests a.phase at run time.
template <int M, int V, int L, bool DIRECT = false, bool STAGE = false, bool PH = true>
__device__ __forceinline__ double patch_step(const StepArgs& a, int s, cx<float>* A,
                                           cx<float>* tws, float* redf, double* redd,
                                           int tid) {
  using P = Px<M, V>;
  constexpr int R = P::ROUNDS, NT = P::NT, LS = P::LS;
  static_assert(M <= NT, "one twiddle per thread");
  constexpr bool XL = Plan<M, V>::XL != 0;
  static_assert(!XL || (M == 64 && Plan<M, V>::R1 == 8 && Plan<M, V>::R2 == 8 && NT == 1024),
                "register-pass plan");
  // LDS slot of tile element (r, c)
  auto at = [](int r, int c) {
    if constexpr (XL) {
      return xl_addr(r, c);
    } else {
      return r * LS + c;
    }
  };
  cx<float> twv{0.f, 0.f};
  if constexpr (STAGE) {
    if (tid < M) twv = ld(a.tw, tid);
  }
  const int4 sl = a.slot[s];
  const int k = sl.x;
  const size_t n = (size_t)a.n;
  const float2* zwin = a.obj + (size_t)sl.y * n + sl.z;
  const float* dk = a.dperm + (size_t)k * M * M;
  // every global load of the patch is issued here, before any dependent work:
  // amplitudes in the order the projection visits them (contiguous across
  // lanes), probe rows as 16-byte pairs, the object window (arbitrary
  // alignment) per pixel
  using CP = ColPass<M, V>;
  cx<float> qc[P::CACHE ? 4 : 1], zc[P::CACHE ? 4 : 1];
  float amp[CP::PTS];
  float ampv[XL ? 8 : 1];
  float q2m = 0.f, z2m = 0.f;
  auto load_amps = [&]() {
#pragma unroll
    for (int it = 0; it < CP::IT; ++it) {
      const int w = tid + it * CP::NT;
      if (CP::ITEMS < CP::NT && w >= CP::ITEMS) break;
      const int line = w % M, g = w / M;
#pragma unroll
      for (int j = 0; j < CP::R1; ++j) amp[it * CP::R1 + j] = dk[(CP::R1 * g + j) * M + line];
    }
  };
  constexpr int AS = Plan<M, V>::AMP;
  constexpr bool DG = Plan<M, V>::DG != 0;
  static_assert(!DG || (!XL && !P::CACHE), "direct gather: LDS plans that reload per round");
  if constexpr (DG) {
    // The exit wave straight into the first (strided) row pass.  Item i = tid + it NT
    // is row i / R1, group g = i % R1, points g + R1 j: the loads of one j cover
    // 64 / R1 rows of a wave, R1 consecutive pixels of each.  The pass runs before the
    // first barrier: a launch that stages its twiddles here (STAGE) reads the pass's
    // W^(g j) from the global table (cache-resident) with the other loads; the kernels
    // that staged them in LDS once at their start (persistent, chain) read them there
    // and hold fewer registers.
    constexpr int R1 = Plan<M, V>::R1, R2 = Plan<M, V>::R2, DIT = M * R1 / NT;
    static_assert(DIT * NT == M * R1, "direct-gather items per thread");
    cx<float> ps[DIT][R2], twr[DIT][R2];
    {
      cx<float> q[DIT][R2], zz[DIT][R2];
#pragma unroll
      for (int it = 0; it < DIT; ++it) {
        const int i = tid + it * NT, row = i / R1, g = i % R1;
#pragma unroll
        for (int j = 0; j < R2; ++j) {
          q[it][j] = ld(a.probe, (size_t)row * M + g + R1 * j);
          zz[it][j] = ld(zwin, (size_t)row * n + g + R1 * j);
        }
        if constexpr (STAGE) {
#pragma unroll
          for (int j = 1; j < R2; ++j) twr[it][j] = ld(a.tw, g * j);
        }
      }
      if constexpr (AS == 0) load_amps();
#pragma unroll
      for (int it = 0; it < DIT; ++it) {
#pragma unroll
        for (int j = 0; j < R2; ++j) {
          q2m = fmaxf(q2m, norm2(q[it][j]));
          z2m = fmaxf(z2m, norm2(zz[it][j]));
          ps[it][j] = mul(q[it][j], zz[it][j]);
        }
      }
    }
    // the strided pass as fft_pass computes it, then the tile to LDS
#pragma unroll
    for (int it = 0; it < DIT; ++it) {
      const int i = tid + it * NT, row = i / R1, g = i % R1;
      dft_small<float, false, R2, M>(ps[it], tws);
#pragma unroll
      for (int j = 1; j < R2; ++j) ps[it][j] = mul_fma(STAGE ? twr[it][j] : tws[g * j], ps[it][j]);
#pragma unroll
      for (int j = 0; j < R2; ++j) A[row * LS + g + R1 * j] = ps[it][j];
    }
  }
#pragma unroll
  for (int rd = 0; rd < (DG ? 0 : R); ++rd) {
    int r0, c0;
    blk_origin<M, V>(tid, rd, r0, c0);
    cx<float> q[4], zz[4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ld_pair(a.probe, (size_t)(r0 + i) * M + c0, q[2 * i], q[2 * i + 1]);
      zz[2 * i] = ld(zwin, (size_t)(r0 + i) * n + c0);
      zz[2 * i + 1] = ld(zwin, (size_t)(r0 + i) * n + c0 + 1);
    }
    // the intensities go out behind the first exit-wave loads, which are needed first
    if constexpr (XL) {
      // waves 8..15: eight amplitudes each, coalesced (element (tid - 512) + 512 j)
      if (rd == 0 && tid >= 512) {
#pragma unroll
        for (int j = 0; j < 8; ++j) ampv[j] = dk[(tid - 512) + 512 * j];
      }
    } else if constexpr (AS == 0) {
      if (rd == 0) load_amps();
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if constexpr (P::CACHE) {
        qc[e] = q[e];
        zc[e] = zz[e];
      }
      q2m = fmaxf(q2m, norm2(q[e]));
      z2m = fmaxf(z2m, norm2(zz[e]));
      A[at(r0 + (e >> 1), c0 + (e & 1))] = mul(q[e], zz[e]);
    }
  }
  if constexpr (STAGE) {
    if (tid < M) tws[tid] = twv;
  }
  // wave maxima go to LDS now; the barriers of the transforms order them
  // before they are read in the per-pixel phase
  wave_max2_to_lds<NT>(q2m, z2m, redf, tid);
  __syncthreads();
  double acc = 0.0;
  if constexpr (XL) {
    // measured amplitudes sqrt(max(d, 0)) in transform order, row stride m + 1
    // (the column phase's reads are then bank-conflict free)
    __shared__ float ampl[M * (M + 1)];
    const int ln = tid & 63, wv = tid >> 6, lo = ln & 7, gi = ln >> 3;
    const int r = 8 * wv + lo, C = 8 * wv + lo;
    cx<float> v[8], w[8];
    if (wv < 8) {
      xl_twiddles(tws, gi, w);
      xl_rows_forward(A, w, r, gi);
    } else {
      xl_stage_amps<M>(ampl, ampv, tid);
    }
    __syncthreads();
    if (wv < 8) {
      // forward column passes, projection, inverse column passes; each lane
      // writes back the elements it read
      xl_cols_forward(A, w, C, gi, v);
      if (PH && a.phase) {
        float2* ph = a.phase + (size_t)k * M * M;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc += (double)project_amp<M>(v[j], ampl[(8 * gi + j) * (M + 1) + C],
                                        ph + (8 * gi + j) * M + C, a.phase_write != 0);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc += (double)project_amp<M>(v[j], ampl[(8 * gi + j) * (M + 1) + C]);
      }
      dft8<float, true>(v);
      xl_transpose8(v);
      xl_strided<true>(v, w);
#pragma unroll
      for (int j = 0; j < 8; ++j) A[xl_addr(gi + 8 * j, C)] = v[j];
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) redd[tid >> 6] = acc;
    __syncthreads();
    if (wv < 8) {
      // inverse row passes; the natural-order result replaces the wave's own rows
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = A[xl_addr(r, 8 * gi + j)];
      dft8<float, true>(v);
      xl_transpose8(v);
      xl_strided<true>(v, w);
#pragma unroll
      for (int j = 0; j < 8; ++j) A[xl_addr(r, gi + 8 * j)] = v[j];
    }
    __syncthreads();
  } else {
    // the forward transform's first three passes (rows, rows, columns); with the
    // direct gather the first one is done
    if constexpr (!DG) {
      fft_pass<float, M, V, false, true, false>(A, tws, tid);
      __syncthreads();
    }
    if constexpr (AS == 1) load_amps();
    fft_pass<float, M, V, false, false, false>(A, tws, tid);
    __syncthreads();
    if constexpr (AS == 2) load_amps();
    fft_pass<float, M, V, false, true, true>(A, tws, tid);
    __syncthreads();
    if constexpr (AS == 3) load_amps();
    // last forward pass, modulus projection, first inverse pass, in registers
    float2* ph = (PH && a.phase) ? a.phase + (size_t)k * M * M : nullptr;
    fft_pass_pair<float, M, V>(A, tid, [&](int e, cx<float>& v) {
      if constexpr (PH) {
        float2* pe = nullptr;
        if (ph) {
          const int w = tid + (e / CP::R1) * CP::NT;
          pe = ph + (CP::R1 * (w / M) + e % CP::R1) * M + w % M;
        }
        acc += (double)project_amp<M>(v, amplitude(amp[e]), pe, a.phase_write != 0);
      } else {
        acc += (double)project_amp<M>(v, amplitude(amp[e]));
      }
    });
    acc = wave_sum(acc);
    if ((tid & 63) == 0) redd[tid >> 6] = acc;
    __syncthreads();
    fft2_inverse_tail<float, M, V>(A, tws, tid);
  }
  float qqmax, zmax;
  lds_max2<NT>(redf, qqmax, zmax);
  pixel_update<M, V, L, DIRECT>(
      a, s, tid,
      [&](int rd, int r0, int c0, cx<float>* q, cx<float>* zz, cx<float>* Rv) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          if constexpr (P::CACHE) {
            q[2 * i] = qc[2 * i];
            q[2 * i + 1] = qc[2 * i + 1];
            zz[2 * i] = zc[2 * i];
            zz[2 * i + 1] = zc[2 * i + 1];
          } else {
            ld_pair(a.probe, (size_t)(r0 + i) * M + c0, q[2 * i], q[2 * i + 1]);
            zz[2 * i] = ld(zwin, (size_t)(r0 + i) * n + c0);
            zz[2 * i + 1] = ld(zwin, (size_t)(r0 + i) * n + c0 + 1);
          }
          Rv[2 * i] = A[at(r0 + i, c0)];
          Rv[2 * i + 1] = A[at(r0 + i, c0 + 1)];
        }
      },
      qqmax, zmax);
  double phi = 0.0;
  if (tid == 0) {
    phi = lds_sum<NT>(redd) / (2.0 * M * M);
    if (a.phi) a.phi[s] = phi;
  }
  __syncthreads();  // LDS is reused by the next slot of a persistent loop
  return phi;
}

// ---------------------------------------------------------------------------
// finalize: FNT threads per work item
//   object tile (item < ntiles): T x T pixels, accumulate the numerators of the
//   overlapping slots in ascending slot order, divide, joint step;
//   probe units: FNT / G pixels x G slot groups (G from the minibatch size),
//   groups combined in a fixed order, then the joint step.
// ---------------------------------------------------------------------------
template <int FNT, int T_>
struct Fin {
  static constexpr int T = T_;
  static constexpr int PER = T * T / FNT;
  static_assert(PER * FNT == T * T && FNT % 256 == 0, "finalize shape");
};
// the finalize shape used inside the persistent kernel (FNT = the plan's NT)
template <int NT>
struct PersistFin {
  static constexpr int T = NT >= 1024 ? 64 : 32;
};

struct FinLds {
  float2 pm[1024];  // probe partial sums of the slot groups
  float pe[1024];
};

// object tiles, then probe units of FNT / G pixels (G slot groups per pixel)
// over an nr x nc object (tile rows of ceil(nc / T) tiles)
template <int M, int FNT, int T>
__host__ __device__ inline int finalize_items(int nr, int nc, int G, int* ntiles_out) {
  const int tiles = ((nr + T - 1) / T) * ((nc + T - 1) / T);
  const int ppu = FNT / G;
  *ntiles_out = tiles;
  return tiles + (M * M + ppu - 1) / ppu;
}

// an empty register barrier: v is taken as written here, so later uses do not
// wait on the load that produced it
__device__ __forceinline__ void settle(int4& v) {
  asm volatile("" : "+v"(v.y), "+v"(v.z));
}

// the lowest set bit of a wave-uniform ballot mask: that lane's slot and window origin
__device__ __forceinline__ bool take_slot(unsigned long long& m, const int4& v, int base, int& slot,
                                          int& ox, int& oy) {
  if (m == 0ull) return false;
  const int bit = __builtin_ctzll(m);
  m &= m - 1ull;
  slot = base + bit;
  ox = __builtin_amdgcn_readlane(v.y, bit);
  oy = __builtin_amdgcn_readlane(v.z, bit);
  return true;
}

template <int M, int FNT, int T>
__device__ __forceinline__ void finalize_item(const StepArgs& a, int item, int ntiles, FinLds& L,
                                              int tid) {
  constexpr int PER = Fin<FNT, T>::PER;
  const int n = a.n, nr = a.nr;  // row stride (columns) and rows of the object
  if (item < ntiles) {
    const int tpr = (n + T - 1) / T;
    const int ty = (item / tpr) * T, tx = (item % tpr) * T;
    // the current object values are needed by the joint step at the end: their
    // loads go out first, beside the slot scan
    cx<float> zold[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * FNT;
      const int y = ty + q / T, x = tx + q % T;
      zold[e] = (a.joint && y < nr && x < n) ? ld(a.obj, (size_t)y * n + x) : cx<float>{0.f, 0.f};
    }
    // Each wave scans the slots itself, 256 at a time (four loads of 64 issued
    // together): a ballot per 64 marks the ones whose window overlaps the tile, and
    // the set bits are taken in ascending order, U per round (every load of a round
    // is issued before its adds; a round may span the four ballots).  No list in LDS,
    // no barrier; the order of the additions is ascending slot order.
    cx<float> accn[PER];
    float accd[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      accn[e] = cx<float>{0.f, 0.f};
      accd[e] = 0.f;
    }
    constexpr int U = FNT >= 1024 ? 2 : 4;
    const int lane = tid & 63;
    for (int s0 = 0; s0 < a.b; s0 += 256) {
      int4 sl0{0, 0, 0, 0}, sl1{0, 0, 0, 0}, sl2{0, 0, 0, 0}, sl3{0, 0, 0, 0};
      const int s = s0 + lane;
      if (s < a.b) sl0 = a.slot[s];
      if (s + 64 < a.b) sl1 = a.slot[s + 64];
      if (s + 128 < a.b) sl2 = a.slot[s + 128];
      if (s + 192 < a.b) sl3 = a.slot[s + 192];
      // the positions are settled here, once: without this the compiler waits for
      // every outstanding load before each lane read of them in the rounds below
      settle(sl0);
      settle(sl1);
      settle(sl2);
      settle(sl3);
      auto overlaps = [&](const int4& v, int j) {
        return j < a.b && !(v.y >= ty + T || v.y + M <= ty || v.z >= tx + T || v.z + M <= tx);
      };
      unsigned long long m0 = __ballot(overlaps(sl0, s)), m1 = __ballot(overlaps(sl1, s + 64)),
                         m2 = __ballot(overlaps(sl2, s + 128)), m3 = __ballot(overlaps(sl3, s + 192));
      // next overlapping slot in ascending order (the masks are wave-uniform)
      auto pop = [&](int& slot, int& ox, int& oy) -> bool {
        return take_slot(m0, sl0, s0, slot, ox, oy) || take_slot(m1, sl1, s0 + 64, slot, ox, oy) ||
               take_slot(m2, sl2, s0 + 128, slot, ox, oy) || take_slot(m3, sl3, s0 + 192, slot, ox, oy);
      };
      while ((m0 | m1 | m2 | m3) != 0ull) {
        cx<float> vn[U][PER];
        float vd[U][PER];
        int sidx[U], ox[U], oy[U];
        // the round's slots first (lane reads of the positions), then its loads: a
        // lane read placed after a load would wait for that load.  cnt (wave-uniform)
        // slots are live; the loops stop there.
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (!pop(sidx[u], ox[u], oy[u])) break;
          ++cnt;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (u >= cnt) break;
          // 32-bit offsets (b m^2 < 2^31): one base address for every load
          const int sb = sidx[u] * (M * M);
#pragma unroll
          for (int e = 0; e < PER; ++e) {
            const int q = tid + e * FNT;
            const int ry = ty + q / T - ox[u], rx = tx + q % T - oy[u];
            const bool in = (unsigned)ry < (unsigned)M && (unsigned)rx < (unsigned)M;
            vn[u][e] = in ? ld32(a.numer, (unsigned)(sb + ry * M + rx)) : cx<float>{0.f, 0.f};
            vd[u][e] = in ? a.Dbuf[(unsigned)(ry * M + rx)] : 0.f;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (u >= cnt) break;
#pragma unroll
          for (int e = 0; e < PER; ++e) {
            accn[e] = add(accn[e], vn[u][e]);
            accd[e] += vd[u][e];
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int q = tid + e * FNT;
      const int y = ty + q / T, x = tx + q % T;
      if (accd[e] >= kMinDivisor && y < nr && x < n) {
        const size_t o = (size_t)y * n + x;
        const cx<float> zp = scale(accn[e], hw_rcp(accd[e]));
        st(a.obj, o, a.joint ? aligned_sqrt(zold[e], zp) : zp);
      }
    }
  } else {
    // probe unit: ppu pixels x G slot groups; group g sums slots [g per, (g + 1) per)
    // in ascending order, then the G partials are added in group order
    const int G = a.pgroups, ppu = FNT / G;
    const int g = tid / ppu, lp = tid - g * ppu;
    const int r = (item - ntiles) * ppu + lp;
    const bool live = a.update_probe && r < M * M;
    const cx<float> qold = (live && g == 0 && a.joint) ? ld(a.probe, r) : cx<float>{0.f, 0.f};
    const int per = (a.b + G - 1) / G;
    const int s_lo = min(a.b, g * per), s_hi = min(a.b, s_lo + per);
    cx<float> mac{0.f, 0.f};
    float eac = 0.f;
    if (live) {
      // U slots per round: the round's loads are all issued before its adds
      constexpr int U = 8;
      for (int s0 = s_lo; s0 < s_hi; s0 += U) {
        cx<float> vm[U];
        float ve[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool in = s0 + u < s_hi;
          const int sl = in ? s0 + u : s_lo;
          const size_t o = (size_t)sl * M * M + r;
          vm[u] = in ? ld(a.pnum, o) : cx<float>{0.f, 0.f};
          ve[u] = in ? (a.pden_slot ? a.pden_slot[sl] : a.pden[o]) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (s0 + u < s_hi) {
            mac = add(mac, vm[u]);
            eac += ve[u];
          }
        }
      }
    }
    L.pm[tid] = make_float2(mac.re, mac.im);
    L.pe[tid] = eac;
    __syncthreads();
    if (g == 0 && live) {
      cx<float> mt = ld(L.pm, lp);
      float et = L.pe[lp];
      for (int k = 1; k < G; ++k) {
        mt = add(mt, ld(L.pm, lp + k * ppu));
        et += L.pe[lp + k * ppu];
      }
      if (et >= kMinDivisor) {
        const cx<float> qp = scale(mt, hw_rcp(et));
        st(a.probe, r, a.joint ? aligned_sqrt(qold, qp) : qp);
      }
    }
    // the batch's sampled misfit: lane j sums the slots j, j + 64, ... (four loads
    // in flight), then the wave sum in its fixed order
    if (item == ntiles && tid < 64 && a.sampled) {
      double t = 0.0;
      for (int s0 = 0; s0 < a.b; s0 += 256) {
        double v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int j = s0 + 64 * c + tid;
          v[c] = j < a.b ? a.phi[j] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) t += v[c];
      }
      t = wave_sum(t);
      if (tid == 0) *a.sampled += t;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// fused path kernels
// ---------------------------------------------------------------------------
template <int M, int NT>
__device__ __forceinline__ void stage_twiddles(const float2* tw, cx<float>* tws, int tid) {
  for (int j = tid; j < M; j += NT) tws[j] = ld(tw, j);
}

// k_patch_step and k_finalize take the slot list, the object and its side (and
// the finalize the slot count) as leading arguments of their own, ahead of the
// argument record, whose copies of them they replace.  The library is built
// with kernel-argument preloading: leading scalar and pointer arguments arrive
// in scalar registers at dispatch, so a kernel's first slot and object loads do
// not wait for a load of its argument record (the record's fields are loaded
// beside them).
template <int M, int V, int L, bool PH>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_patch_step(const int4* slot, float2* obj,
                                                                 int n, StepArgs rec) {
  StepArgs a = rec;
  a.slot = slot;
  a.obj = obj;
  a.n = n;
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ float redf[32];
  __shared__ double redd[16];
  const int tid = threadIdx.x;
  patch_step<M, V, L, false, true, PH>(a, blockIdx.x, A, tws, redf, redd, tid);
}

// ---------------------------------------------------------------------------
// many independent reconstructions in one launch: block b serves work item
// work[b] = (instance argument record, slot or finalize item); every
// instance keeps its own state, data and workspace, so the arithmetic is the
// single-instance arithmetic
// ---------------------------------------------------------------------------
template <int M, int V, int L, bool PH>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_patch_step_multi(const StepArgs* args,
                                                                     const int2* work) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ float redf[32];
  __shared__ double redd[16];
  const int tid = threadIdx.x;
  const int2 w = work[blockIdx.x];
  const StepArgs a = args[w.x];
  patch_step<M, V, L, false, true, PH>(a, w.y, A, tws, redf, redd, tid);
}

template <int M, int F>
__global__ __launch_bounds__(FinShape<F>::FNT) void k_finalize(const int4* slot, float2* obj, int n,
                                                               int b, StepArgs rec, int ntiles) {
  StepArgs a = rec;
  a.slot = slot;
  a.obj = obj;
  a.n = n;
  a.b = b;
  constexpr int FNT = FinShape<F>::FNT, T = FinShape<F>::T;
  __shared__ FinLds L;
  const int tid = threadIdx.x;
  int item = blockIdx.x;
  if constexpr (FinShape<F>::BANDED) {
    // Blocks i < ntiles with i mod X = x are the k-th (k = i / X) of the q + (x < r)
    // blocks on XCD x (ntiles = q X + r); they take band x, tiles x q + min(x, r) + k.
    constexpr int X = kDispatchXcds;
    if (item < ntiles) {
      const int q = ntiles / X, r = ntiles % X, x = item % X;
      item = x * q + min(x, r) + item / X;
    }
  } else if constexpr (FinShape<F>::ORDER == 2) {
    if (item < ntiles) item = rows_per_xcd_tile(item, ntiles, (n + T - 1) / T);
  }
  finalize_item<M, FNT, T>(a, item, ntiles, L, tid);
}

template <int M, int F>
__global__ __launch_bounds__(FinShape<F>::FNT) void k_finalize_multi(const StepArgs* args,
                                                                    const int2* work) {
  constexpr int FNT = FinShape<F>::FNT, T = FinShape<F>::T;
  __shared__ FinLds L;
  const int tid = threadIdx.x;
  const int2 w = work[blockIdx.x];
  const StepArgs a = args[w.x];
  int ntiles;
  finalize_items<M, FNT, T>(a.nr, a.n, a.pgroups, &ntiles);
  finalize_item<M, FNT, T>(a, w.y, ntiles, L, tid);
}

// Grid-wide barrier for the persistent kernel (all workgroups co-resident by
// cooperative launch).  Each wave waits until its own global stores have
// reached L2; then one lane per workgroup releases at agent scope (L2
// write-back, so other XCDs see the data), arrives on a monotonic counter,
// waits for the target and acquires (stale lines dropped from this CU's L1 and
// this XCD's L2) before the workgroup proceeds.  A bounded spin (spin_limit polls)
// turns a lost arrival into an error flag instead of a hang: *err is set with a
// system-scope store (it may live in host memory, where the host reads it at its
// next call) and the workgroup goes on.
__device__ __forceinline__ void grid_barrier(unsigned* ctr, unsigned target, int* err,
                                             unsigned spin_limit) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(4);
      if (++spins > spin_limit) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// persistent epoch: every minibatch of a sweep in one cooperative launch
template <int M, int V, int L, bool PH>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_epoch_persistent(StepArgs a, int n_pos, int B,
                                                                     int ntiles, int nitems,
                                                                     unsigned* bar,
                                                                     unsigned bar_base, int* err,
                                                                     unsigned spin_limit) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ float redf[32];
  __shared__ double redd[16];
  __shared__ FinLds FL;
  constexpr int NT = Plan<M, V>::NT, FT = PersistFin<NT>::T;
  const int tid = threadIdx.x;
  stage_twiddles<M, NT>(a.tw, tws, tid);
  __syncthreads();
  const int4* slots = a.slot;
  unsigned target = bar_base;
  for (int start = 0; start < n_pos; start += B) {
    StepArgs x = a;
    x.slot = slots + start;
    x.b = min(B, n_pos - start);
    for (int s = blockIdx.x; s < x.b; s += gridDim.x)
      patch_step<M, V, L, false, false, PH>(x, s, A, tws, redf, redd, tid);
    target += gridDim.x;
    grid_barrier(bar, target, err, spin_limit);
    for (int item = blockIdx.x; item < nitems; item += gridDim.x)
      finalize_item<M, NT, FT>(x, item, ntiles, FL, tid);
    target += gridDim.x;
    grid_barrier(bar, target, err, spin_limit);
  }
}

// Sequential sweep of minibatch-1 steps in one workgroup (the paper's literal
// order: each step sees the previous step's object and probe).  No grid-wide
// synchronisation: every step touches only its own window and the probe, and the
// workgroup barrier at the end of each step orders it before the next.  The
// sampled misfit accumulates exactly as the finalize adds it.
template <int M, int V, int L, bool PH>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_sweep_chain(StepArgs a, int n_steps) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ float redf[32];
  __shared__ double redd[16];
  const int tid = threadIdx.x;
  stage_twiddles<M, Plan<M, V>::NT>(a.tw, tws, tid);
  __syncthreads();
  const int4* slots = a.slot;
  // the running sum stays in a register of thread 0 (the finalize's order:
  // sampled <- sampled + (0 + phi) after every step), stored once at the end
  double sampled = (tid == 0 && a.sampled) ? *a.sampled : 0.0;
  for (int step = 0; step < n_steps; ++step) {
    StepArgs x = a;
    x.slot = slots + step;
    x.b = 1;
    const double phi = patch_step<M, V, L, true, false, PH>(x, 0, A, tws, redf, redd, tid);
    double t = 0.0;
    t += phi;
    sampled += t;
  }
  if (tid == 0 && a.sampled) *a.sampled = sampled;
}

// ---------------------------------------------------------------------------
// plain path: one launch per stage, intermediates in HBM
// ---------------------------------------------------------------------------
template <int M, int V>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_probe_prep(StepArgs a) {
  __shared__ float redf[32];
  const int tid = threadIdx.x;
  float q2m = 0.f, dummy = 0.f;
  for (int r = tid; r < M * M; r += Plan<M, V>::NT) q2m = fmaxf(q2m, norm2(ld(a.probe, r)));
  block_max2<Plan<M, V>::NT>(q2m, dummy, redf, tid);
  if (tid == 0) a.qqmax[0] = q2m;
}

template <int M, int V>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_gather(StepArgs a) {
  __shared__ float redf[32];
  constexpr int PX = Px<M, V>::PX;
  const int tid = threadIdx.x, s = blockIdx.x;
  const float2* zwin = a.obj + (size_t)a.slot[s].y * a.n + a.slot[s].z;
  float z2m = 0.f, dummy = 0.f;
#pragma unroll
  for (int e = 0; e < PX; ++e) {
    int r, c;
    pix_rc<M, V>(tid, e, r, c);
    const cx<float> q = ld(a.probe, (size_t)r * M + c);
    const cx<float> zz = ld(zwin, (size_t)r * a.n + c);
    z2m = fmaxf(z2m, norm2(zz));
    st(a.stack, (size_t)s * M * M + r * M + c, mul(q, zz));
  }
  block_max2<Plan<M, V>::NT>(z2m, dummy, redf, tid);
  if (tid == 0) a.zmax[s] = z2m;
}

template <int M, int V, bool INV>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_fft(StepArgs a) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  constexpr int NT = Plan<M, V>::NT, LS = lds_stride<M>();
  const int tid = threadIdx.x;
  float2* X = a.stack + (size_t)blockIdx.x * M * M;
  stage_twiddles<M, NT>(a.tw, tws, tid);
  for (int e = tid; e < M * M; e += NT) A[(e / M) * LS + e % M] = ld(X, e);
  __syncthreads();
  if (INV) fft2_inverse<float, M, V>(A, tws, tid);
  else fft2_forward<float, M, V>(A, tws, tid);
  for (int e = tid; e < M * M; e += NT) st(X, e, A[(e / M) * LS + e % M]);
}

template <int M, int V>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_project(StepArgs a) {
  __shared__ double redd[16];
  constexpr int PX = Px<M, V>::PX, NT = Px<M, V>::NT;
  const int tid = threadIdx.x, s = blockIdx.x;
  float2* X = a.stack + (size_t)s * M * M;
  const float* dk = a.dperm + (size_t)a.slot[s].x * M * M;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < PX; ++e) {
    int r, c;
    pix_rc<M, V>(tid, e, r, c);
    const size_t o = (size_t)r * M + c;
    cx<float> P = ld(X, o);
    float2* ph = a.phase ? a.phase + (size_t)a.slot[s].x * M * M + o : nullptr;
    acc += (double)project_px<M>(P, dk[o], ph, a.phase_write != 0);
    st(X, o, P);
  }
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0 && a.phi) a.phi[s] = tot / (2.0 * M * M);
}

template <int M, int V, int L>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_numerators(StepArgs a) {
  const int tid = threadIdx.x, s = blockIdx.x;
  const size_t n = (size_t)a.n;
  const float2* zwin = a.obj + (size_t)a.slot[s].y * n + a.slot[s].z;
  const float2* Rg = a.stack + (size_t)s * M * M;
  pixel_update<M, V, L>(
      a, s, tid,
      [&](int rd, int r0, int c0, cx<float>* q, cx<float>* zz, cx<float>* Rv) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          ld_pair(a.probe, (size_t)(r0 + i) * M + c0, q[2 * i], q[2 * i + 1]);
          zz[2 * i] = ld(zwin, (size_t)(r0 + i) * n + c0);
          zz[2 * i + 1] = ld(zwin, (size_t)(r0 + i) * n + c0 + 1);
          ld_pair(Rg, (size_t)(r0 + i) * M + c0, Rv[2 * i], Rv[2 * i + 1]);
        }
      },
      a.qqmax[0], a.zmax[s]);
}

// ---------------------------------------------------------------------------
// misfit and gradient
// ---------------------------------------------------------------------------
// Misfit term Phi_k = sum (|F(Q . z_k)| - a_k)^2 / (2 m^2) of one pattern (Eq. 1, Parseval
// form), returned in thread 0.  The twiddles are already in tws (the caller synchronises
// after staging them).  INT(row, col) is the measured intensity at transform-order position
// (row, col): dk[row * M + col] for intensities laid out in the plan's transform order, or
// d[freq(row) * M + freq(col)] for intensities in natural order.
template <int M, int V, class INT>
__device__ __forceinline__ double misfit_pattern(const float2* obj, int n, const float2* probe,
                                                 int2 pk, INT intensity, cx<float>* A,
                                                 const cx<float>* tws, double* redd, int tid) {
  constexpr int PX = Px<M, V>::PX, NT = Px<M, V>::NT, LS = Px<M, V>::LS;
#pragma unroll
  for (int e = 0; e < PX; ++e) {
    int r, c;
    pix_rc<M, V>(tid, e, r, c);
    A[r * LS + c] = mul(ld(probe, (size_t)r * M + c), ld(obj, (size_t)(pk.x + r) * n + pk.y + c));
  }
  // the intensities in the order the last pass visits them
  using CP = ColPass<M, V>;
  float dv[CP::PTS];
#pragma unroll
  for (int it = 0; it < CP::IT; ++it) {
    const int w = tid + it * CP::NT;
    if (CP::ITEMS < CP::NT && w >= CP::ITEMS) break;
    const int line = w % M, g = w / M;
#pragma unroll
    for (int j = 0; j < CP::R1; ++j) dv[it * CP::R1 + j] = intensity(CP::R1 * g + j, line);
  }
  __syncthreads();
  fft_pass<float, M, V, false, true, false>(A, tws, tid);
  __syncthreads();
  fft_pass<float, M, V, false, false, false>(A, tws, tid);
  __syncthreads();
  fft_pass<float, M, V, false, true, true>(A, tws, tid);
  __syncthreads();
  // the last pass hands each transformed value to the misfit term, in registers
  double acc = 0.0;
  fft_pass_last<float, M, V>(A, tid, [&](int e, cx<float> P) {
    acc += (double)project_px<M>(P, dv[e]);
  });
  const double tot = block_sum<NT>(acc, redd, tid);
  return tot / (2.0 * M * M);
}

template <int M, int V>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_misfit(const float2* obj, int n,
                                                        const float2* probe, const float* dperm,
                                                        const int2* pos, const int4* slot,
                                                        const float2* tw, double* phi_all,
                                                        int by_pattern) {
  __shared__ cx<float> A[M * lds_stride<M>()];
  __shared__ cx<float> tws[M];
  __shared__ double redd[16];
  constexpr int NT = Px<M, V>::NT;
  // all patterns (slot == nullptr: block k is pattern k) or the patterns of a slot list;
  // the term goes to the block's place, or with by_pattern to its pattern's index
  const int tid = threadIdx.x;
  const int k = slot ? slot[blockIdx.x].x : (int)blockIdx.x;
  const int2 pk = slot ? make_int2(slot[blockIdx.x].y, slot[blockIdx.x].z) : pos[k];
  const float* dk = dperm + (size_t)k * M * M;
  stage_twiddles<M, NT>(tw, tws, tid);
  const double phi = misfit_pattern<M, V>(obj, n, probe, pk,
                                          [&](int r, int c) { return dk[r * M + c]; }, A, tws,
                                          redd, tid);
  if (tid == 0) phi_all[by_pattern ? k : (int)blockIdx.x] = phi;
}

// The misfit term of one pattern at m = 128 (splits 16 x 8 and 8 x 16) with two
// workgroups per CU: 512 threads, and half the transformed tile in LDS at a time (S:
// 128 rows of 64, row stride 65), the other half held in registers.  The rows go in two
// chunks of 64: the strided row pass loads its exit wave straight from memory (item
// (row, g) its points g + R1 j), the contiguous row pass leaves each thread 16 values of
// each chunk in registers.  With the 16 x 8 split a thread's contiguous item is one
// 16-point run, and the second chunk's item has the first one's group with bit 2
// flipped, so the thread holds one run in columns 0..63 and one in 64..127; with 8 x 16
// a thread has two 8-point items per chunk, one in each column half.  Then the column
// passes of columns 0..63 in LDS, and those of 64..127 once the other runs are written
// in.  Every DFT, twiddle product and misfit term is the one the plan's LDS passes
// compute (misfit_pattern), so the terms are bitwise the same; only the order of the
// pattern's FP64 sum differs.  The caller has staged the twiddles in tws and
// synchronised; INT as in misfit_pattern.
template <int M, int V>
struct HalfMisfit {
  static constexpr int R1 = Plan<M, V>::R1, R2 = Plan<M, V>::R2;
  static constexpr bool value = M == 128 && ((R1 == 16 && R2 == 8) || (R1 == 8 && R2 == 16));
  static constexpr int NT = 512, H = M / 2;
  static constexpr int LR = M + 1;  // row chunk: 64 rows of 128, stride 129
  static constexpr int LC = H + 1;  // column half: 128 rows of 64, stride 65
  static constexpr int LDS = M * LC;
  static_assert(H * LR <= M * LC, "row chunk fits the column-half buffer");
};

template <int M, int V, class INT>
__device__ __forceinline__ double misfit_pattern_half(const float2* obj, int n, const float2* probe,
                                                      int2 pk, INT intensity, cx<float>* S,
                                                      const cx<float>* tws, double* redd, int tid) {
  using HM = HalfMisfit<M, V>;
  constexpr int NTH = HM::NT, H = HM::H, LR = HM::LR, LC = HM::LC, R1 = HM::R1, R2 = HM::R2;
  static_assert(HM::value, "m = 128, split 16 x 8 or 8 x 16");
  // items per thread of the strided (R2 points) and contiguous (R1 points) passes over
  // 64 lines
  constexpr int IT1 = H * R1 / NTH, IT2 = H * R2 / NTH;
  static_assert(IT1 * NTH == H * R1 && IT2 * NTH == H * R2 && IT2 * R1 == 16, "items per thread");
  const int rl = tid % H, gq = tid / H;  // contiguous row items: row rl of the chunk, group gq (+ 8 it)
  cx<float> hold[2][IT2][R1];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // strided row pass over the chunk's 64 rows
#pragma unroll
    for (int it = 0; it < IT1; ++it) {
      const int w = tid + it * NTH;
      const int r = w / R1, g = w % R1;
      const int row = h * H + r;
      cx<float> v[R2];
#pragma unroll
      for (int j = 0; j < R2; ++j) {
        const int c = g + R1 * j;
        v[j] = mul(ld(probe, (size_t)row * M + c), ld(obj, (size_t)(pk.x + row) * n + pk.y + c));
      }
      dft_small<float, false, R2, M>(v, tws);
#pragma unroll
      for (int j = 1; j < R2; ++j) v[j] = mul_fma(tws[g * j], v[j]);
#pragma unroll
      for (int j = 0; j < R2; ++j) S[r * LR + g + R1 * j] = v[j];
    }
    __syncthreads();
    // contiguous row pass: row rl, group gq + 8 it (16 x 8: gq, or gq ^ 4 in chunk 1)
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int g = IT2 == 1 ? (gq ^ (h * (R2 / 2))) : gq + 8 * it;
#pragma unroll
      for (int j = 0; j < R1; ++j) hold[h][it][j] = S[rl * LR + R1 * g + j];
      dft_small<float, false, R1, M>(hold[h][it], nullptr);
    }
    __syncthreads();
  }
  // 16 x 8: the run in columns 0..63 (A) and the one in 64..127 (B)
  const bool first = gq < R2 / 2;
  const int rowA = first ? rl : H + rl, rowB = first ? H + rl : rl;
  const int cA = R1 * (gq & (R2 / 2 - 1));  // column of the run within its half
  cx<float> hB[R1];
  double acc = 0.0;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if constexpr (IT2 == 1) {
      if (half == 0) {
#pragma unroll
        for (int j = 0; j < R1; ++j) {
          S[rowA * LC + cA + j] = first ? hold[0][0][j] : hold[1][0][j];
          hB[j] = first ? hold[1][0][j] : hold[0][0][j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < R1; ++j) S[rowB * LC + cA + j] = hB[j];
      }
    } else {
      // 8 x 16: item it of each chunk lies in column half it (columns 8 gq + j of it)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < R1; ++j) S[(h * H + rl) * LC + R1 * gq + j] = hold[h][half][j];
    }
    // this half's intensities, in the order the last pass visits them
    float dv[IT2][R1];
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int w = tid + it * NTH, line = w % H, g = w / H;
#pragma unroll
      for (int j = 0; j < R1; ++j) dv[it][j] = intensity(R1 * g + j, half * H + line);
    }
    __syncthreads();
    // strided column pass over the half's 64 columns
#pragma unroll
    for (int it = 0; it < IT1; ++it) {
      const int w = tid + it * NTH;
      const int ln = w % H, g = w / H;
      cx<float> v[R2];
#pragma unroll
      for (int j = 0; j < R2; ++j) v[j] = S[(g + R1 * j) * LC + ln];
      dft_small<float, false, R2, M>(v, tws);
#pragma unroll
      for (int j = 1; j < R2; ++j) v[j] = mul_fma(tws[g * j], v[j]);
#pragma unroll
      for (int j = 0; j < R2; ++j) S[(g + R1 * j) * LC + ln] = v[j];
    }
    __syncthreads();
    // contiguous column pass with the misfit terms
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int w = tid + it * NTH, line = w % H, g = w / H;
      cx<float> v[R1];
#pragma unroll
      for (int j = 0; j < R1; ++j) v[j] = S[(R1 * g + j) * LC + line];
      dft_small<float, false, R1, M>(v, nullptr);
#pragma unroll
      for (int j = 0; j < R1; ++j) acc += (double)project_px<M>(v[j], dv[it][j]);
    }
    __syncthreads();
  }
  const double tot = block_sum<NTH>(acc, redd, tid);
  return tot / (2.0 * M * M);
}

// Two workgroups per CU need at most 128 VGPRs (four waves per SIMD).  The 16 x 8 split
// takes 125 as built; asking the compiler for four waves per SIMD outright makes it use
// all 128 and spill, so its bound states only a floor of two waves.  The 8 x 16 split
// (16-point strided passes) would take 164 unbounded and fits 128 without spilling
// when asked for four waves.
template <int M, int V>
__global__ __launch_bounds__(512, (Plan<M, V>::R2 == 16 ? 4 : 2)) void k_misfit_half(const float2* obj, int n,
                                                        const float2* probe, const float* dperm,
                                                        const int2* pos, const int4* slot,
                                                        const float2* tw, double* phi_all,
                                                        int by_pattern) {
  using HM = HalfMisfit<M, V>;
  __shared__ cx<float> S[HM::LDS];
  __shared__ cx<float> tws[M];
  __shared__ double redd[16];
  const int tid = threadIdx.x;
  const int k = slot ? slot[blockIdx.x].x : (int)blockIdx.x;
  const int2 pk = slot ? make_int2(slot[blockIdx.x].y, slot[blockIdx.x].z) : pos[k];
  const float* dk = dperm + (size_t)k * M * M;
  stage_twiddles<M, HM::NT>(tw, tws, tid);
  __syncthreads();
  const double phi = misfit_pattern_half<M, V>(obj, n, probe, pk,
                                               [&](int r, int c) { return dk[r * M + c]; }, S, tws,
                                               redd, tid);
  if (tid == 0) phi_all[by_pattern ? k : (int)blockIdx.x] = phi;
}

// Quadratic surrogate of Eq. 3 for the slots of a batch: 1/2 ||Q . z_k - R_k||^2 with the
// current state (Q, z) and revised exit waves R_k held in a.stack (frozen at an earlier
// iterate).  FP32 differences, FP64 sum of their squared magnitudes.
template <int M, int V>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_surrogate(StepArgs a, double* terms) {
  __shared__ double redd[16];
  constexpr int PX = Px<M, V>::PX, NT = Px<M, V>::NT;
  const int tid = threadIdx.x, s = blockIdx.x;
  const int4 sl = a.slot[s];
  const float2* zwin = a.obj + (size_t)sl.y * a.n + sl.z;
  const float2* Rg = a.stack + (size_t)s * M * M;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < PX; ++e) {
    int r, c;
    pix_rc<M, V>(tid, e, r, c);
    const cx<float> d = sub(mul(ld(a.probe, (size_t)r * M + c), ld(zwin, (size_t)r * a.n + c)),
                            ld(Rg, (size_t)r * M + c));
    acc += (double)d.re * (double)d.re + (double)d.im * (double)d.im;
  }
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0) terms[s] = 0.5 * tot;
}

template <typename T>
__device__ __forceinline__ cx<T> ldT(const void* p, size_t i) {
  return reinterpret_cast<const cx<T>*>(p)[i];
}
template <typename T>
__device__ __forceinline__ void stT(void* p, size_t i, cx<T> v) {
  reinterpret_cast<cx<T>*>(p)[i] = v;
}

template <typename T, int M, int V>
__global__ __launch_bounds__((Plan<M, V>::NT)) void k_grad_patch(GradArgs g, int k0) {
  __shared__ cx<T> A[M * lds_stride<M>()];
  __shared__ cx<T> tws[M];
  __shared__ double redd[16];
  constexpr int PX = Px<M, V>::PX, NT = Px<M, V>::NT, LS = Px<M, V>::LS;
  const int tid = threadIdx.x, s = blockIdx.x, k = k0 + s;
  const int2 pk = g.pos[k];
  const size_t n = (size_t)g.n;
  for (int j = tid; j < M; j += NT) tws[j] = ldT<T>(g.tw, j);
#pragma unroll
  for (int e = 0; e < PX; ++e) {
    int r, c;
    pix_rc<M, V>(tid, e, r, c);
    A[r * LS + c] = mul(ldT<T>(g.probe, (size_t)r * M + c), ldT<T>(g.obj, (pk.x + r) * n + pk.y + c));
  }
  // the intensities in the order the middle pass visits them (see patch_step)
  using CP = ColPass<M, V>;
  const float* dk = g.dperm + (size_t)k * M * M;
  float dv[CP::PTS];
#pragma unroll
  for (int it = 0; it < CP::IT; ++it) {
    const int w = tid + it * CP::NT;
    if (CP::ITEMS < CP::NT && w >= CP::ITEMS) break;
    const int line = w % M, gg = w / M;
#pragma unroll
    for (int j = 0; j < CP::R1; ++j) dv[it * CP::R1 + j] = dk[(CP::R1 * gg + j) * M + line];
  }
  __syncthreads();
  fft_pass<T, M, V, false, true, false>(A, tws, tid);
  __syncthreads();
  fft_pass<T, M, V, false, false, false>(A, tws, tid);
  __syncthreads();
  fft_pass<T, M, V, false, true, true>(A, tws, tid);
  __syncthreads();
  // last forward pass, residual in Fourier space, first inverse pass, in registers:
  // Psi - Psi' = (|Psi| - a) Psi/|Psi|, or -a where Psi = 0
  const T inv_m2 = T(1) / T(M * M);
  double acc = 0.0;
  fft_pass_pair<T, M, V>(A, tid, [&](int e, cx<T>& P) {
    const T amp = sqrt(fmax(T(dv[e]), T(0)));
    const T mag = sqrt(norm2(P));
    const T diff = mag - amp;
    acc += (double)diff * (double)diff;
    const cx<T> E = mag > T(0) ? scale(P, diff / mag) : cx<T>{-amp, T(0)};
    P = scale(E, inv_m2);
  });
  __syncthreads();
  fft2_inverse_tail<T, M, V>(A, tws, tid);
  const size_t base = (size_t)s * M * M;
#pragma unroll
  for (int e = 0; e < PX; ++e) {
    int r, c;
    pix_rc<M, V>(tid, e, r, c);
    const cx<T> ev = A[r * LS + c];
    const cx<T> q = ldT<T>(g.probe, (size_t)r * M + c);
    const cx<T> zz = ldT<T>(g.obj, (pk.x + r) * n + pk.y + c);
    stT<T>(g.gz_slots, base + r * M + c, cmulc(q, ev));
    stT<T>(g.gq_slots, base + r * M + c, cmulc(zz, ev));
  }
  const double tot = block_sum<NT>(acc, redd, tid);
  if (tid == 0) g.phi_all[k] = tot / (2.0 * M * M);
}

// Deterministic reductions of the per-pattern gradient slots.  Both split a
// chunk's patterns into contiguous groups summed in parallel (ascending order
// inside a group) and add the group partials in group order, with several loads
// in flight per round; the order depends only on the chunk, not on the launch.
constexpr int kGradTile = 16;   // object gradient tiles kGradTile^2
constexpr int kGradZGroups = 4; // pattern groups per object tile (one per 256 threads)
constexpr int kGradQGroups = 16;  // pattern groups per probe pixel

__device__ __forceinline__ void settle2(int2& v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y));
}

// object gradient: tile `tile` of kGradTile^2 pixels, kGradZGroups x 256 threads
template <typename T, int M>
__device__ __forceinline__ void grad_scatter_tile(const GradArgs& g, int k0, int cnt, int first,
                                                  int tile, cx<T>* part, int tid) {
  constexpr int TS = kGradTile, GS = kGradZGroups, U = 8;
  static_assert(TS * TS == 256, "one pixel per thread of a group");
  const int gi = tid >> 8, q = tid & 255, lane = tid & 63, n = g.n, nr = g.nr;
  const int tpr = (n + TS - 1) / TS;
  const int ty = (tile / tpr) * TS, tx = (tile % tpr) * TS;
  const int y = ty + q / TS, x = tx + q % TS;
  const int per = (cnt + GS - 1) / GS, lo = min(cnt, gi * per), hi = min(cnt, lo + per);
  cx<T> acc{T(0), T(0)};
  for (int s0 = lo; s0 < hi; s0 += 64) {
    const int sj = s0 + lane;
    int2 p{0, 0};
    if (sj < hi) p = g.pos[k0 + sj];
    settle2(p);
    const bool ov = sj < hi && !(p.x >= ty + TS || p.x + M <= ty || p.y >= tx + TS || p.y + M <= tx);
    unsigned long long m = __ballot(ov);
    while (m != 0ull) {
      int sl[U], ox[U], oy[U];
      int c = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (m == 0ull) break;
        const int bit = __builtin_ctzll(m);
        m &= m - 1ull;
        sl[u] = s0 + bit;
        ox[u] = __builtin_amdgcn_readlane(p.x, bit);
        oy[u] = __builtin_amdgcn_readlane(p.y, bit);
        ++c;
      }
      __builtin_amdgcn_sched_barrier(0);
      cx<T> v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (u >= c) break;
        const int ry = y - ox[u], rx = x - oy[u];
        const bool in = (unsigned)ry < (unsigned)M && (unsigned)rx < (unsigned)M;
        v[u] = in ? ldT<T>(g.gz_slots, (size_t)sl[u] * M * M + ry * M + rx) : cx<T>{T(0), T(0)};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (u >= c) break;
        acc = add(acc, v[u]);
      }
    }
  }
  if (gi > 0) part[(gi - 1) * TS * TS + q] = acc;
  __syncthreads();
  if (gi == 0 && y < nr && x < n) {
#pragma unroll
    for (int k = 1; k < GS; ++k) acc = add(acc, part[(k - 1) * TS * TS + q]);
    const size_t o = (size_t)y * n + x;
    stT<T>(g.gobj, o, first ? acc : add(ldT<T>(g.gobj, o), acc));
  }
}

// probe gradient: unit `unit` of 256 threads, 256 / kGradQGroups pixels x kGradQGroups
// pattern groups (part: the unit's 256 partial sums; every thread of the block calls
// this once, for the barrier)
template <typename T, int M>
__device__ __forceinline__ void grad_probe_unit(const GradArgs& g, int cnt, int first, int unit,
                                                cx<T>* part, int tid) {
  constexpr int G = kGradQGroups, PPU = 256 / G, U = 8;
  const int gi = tid / PPU, lp = tid % PPU;
  const int r = unit * PPU + lp;
  const bool live = r < M * M;
  const int per = (cnt + G - 1) / G, lo = min(cnt, gi * per), hi = min(cnt, lo + per);
  cx<T> acc{T(0), T(0)};
  if (live) {
    for (int s0 = lo; s0 < hi; s0 += U) {
      cx<T> v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        v[u] = s0 + u < hi ? ldT<T>(g.gq_slots, (size_t)(s0 + u) * M * M + r) : cx<T>{T(0), T(0)};
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (s0 + u < hi) acc = add(acc, v[u]);
    }
  }
  part[tid] = acc;
  __syncthreads();
  if (gi == 0 && live) {
    cx<T> t = part[lp];
#pragma unroll
    for (int k = 1; k < G; ++k) t = add(t, part[lp + k * PPU]);
    stT<T>(g.gprobe, r, first ? t : add(ldT<T>(g.gprobe, r), t));
  }
}

// the object and probe reductions of one chunk in one launch: blocks [0, tiles) take
// object tiles, the others four probe units each (256 threads per unit)
constexpr int kGradUnitsPerBlock = kGradZGroups;
inline int grad_tiles(const GradArgs& g) {
  return ((g.nr + kGradTile - 1) / kGradTile) * ((g.n + kGradTile - 1) / kGradTile);
}
inline int grad_probe_blocks(int m) {
  const int units = (m * m + 256 / kGradQGroups - 1) / (256 / kGradQGroups);
  return (units + kGradUnitsPerBlock - 1) / kGradUnitsPerBlock;
}
template <typename T, int M>
__global__ __launch_bounds__(256 * kGradZGroups) void k_grad_reduce(GradArgs g, int k0, int cnt,
                                                                     int first, int tiles) {
  __shared__ cx<T> part[256 * kGradZGroups];
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < tiles)
    grad_scatter_tile<T, M>(g, k0, cnt, first, blockIdx.x, part, tid);
  else
    grad_probe_unit<T, M>(g, cnt, first,
                          ((int)blockIdx.x - tiles) * kGradUnitsPerBlock + (tid >> 8),
                          part + (tid & ~255), tid & 255);
}

// ---------------------------------------------------------------------------
// init helpers
// ---------------------------------------------------------------------------
template <int M, int V>
__global__ __launch_bounds__(256) void k_layout(const float* d, float* dperm, double* sums,
                                                int* bad) {
  __shared__ double redd[16];
  const int tid = threadIdx.x, k = blockIdx.x;
  const float* src = d + (size_t)k * M * M;
  float* dst = dperm + (size_t)k * M * M;
  double acc = 0.0;
  int nonfinite = 0;
  for (int e = tid; e < M * M; e += 256) {
    const float v = src[freq_of_pos<M, V>(e / M) * M + freq_of_pos<M, V>(e % M)];
    dst[e] = fmaxf(v, 0.f);  // amplitude() takes the root of this without a test
    nonfinite |= !isfinite(v);
    acc += (double)v;
  }
  if (nonfinite) atomicOr(bad, 1);
  const double tot = block_sum<256>(acc, redd, tid);
  if (tid == 0) sums[k] = tot;
}

template <int M>
__global__ __launch_bounds__(256) void k_normalize(float2* probe, double dp_avg, int* zero_flag) {
  __shared__ double redd[16];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int r = tid; r < M * M; r += 256) {
    const float2 v = probe[r];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double tot = block_sum<256>(acc, redd, tid);
  if (tot == 0.0) {
    if (tid == 0) zero_flag[0] = 1;
    return;
  }
  const float sc = (float)(dp_avg / sqrt(tot));
  for (int r = tid; r < M * M; r += 256) {
    const float2 v = probe[r];
    probe[r] = make_float2(v.x * sc, v.y * sc);
  }
}


// ---------------------------------------------------------------------------
// launchers: Launchers<M> (declared in launch.hpp) for one probe side, with
// run-time plan / level / finalize-shape choice mapped onto instantiations
// ---------------------------------------------------------------------------
template <int N>
using IC = std::integral_constant<int, N>;

template <int M, class Fn>
hipError_t with_plan(int v, Fn&& fn) {
  switch (v) {
    case 0: return fn(IC<0>{});
    case 1: if constexpr (PlanCount<M>::value > 1) return fn(IC<1>{}); break;
    case 2: if constexpr (PlanCount<M>::value > 2) return fn(IC<2>{}); break;
    case 3: if constexpr (PlanCount<M>::value > 3) return fn(IC<3>{}); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

// PH of the patch kernels: compiled without the phase memory when a.phase is null
template <class Fn>
hipError_t with_phase(const StepArgs& a, Fn&& fn) {
  if (a.phase) return fn(std::true_type{});
  return fn(std::false_type{});
}

template <class Fn>
hipError_t with_levels(int L, Fn&& fn) {
  switch (L) {
    case 1: return fn(IC<1>{});
    case 2: return fn(IC<2>{});
    case 3: return fn(IC<3>{});
    default: return hipErrorInvalidValue;
  }
}

template <class Fn>
hipError_t with_fin(int f, Fn&& fn) {
  switch (f) {
    case 0: return fn(IC<0>{});
    case 1: return fn(IC<1>{});
    case 2: return fn(IC<2>{});
    case 3: return fn(IC<3>{});
    case 4: return fn(IC<4>{});
    case 5: return fn(IC<5>{});
    case 6: return fn(IC<6>{});
    case 7: return fn(IC<7>{});
    case 8: return fn(IC<8>{});
    case 9: return fn(IC<9>{});
    case 10: return fn(IC<10>{});
    case 11: return fn(IC<11>{});
    default: return hipErrorInvalidValue;
  }
}

// With timing events the launch goes through hipExtLaunchKernel, which
// timestamps the kernel's own execution (the dispatch is not included).
template <int M>
hipError_t Launchers<M>::patch_step(int v, int L, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                                    hipEvent_t e1) {
  return with_plan<M>(v, [&](auto vc) {
    return with_levels(L, [&](auto lc) {
      return with_phase(a, [&](auto pc) {
        constexpr int V = decltype(vc)::value, LV = decltype(lc)::value, NT = Plan<M, V>::NT;
        constexpr bool PH = decltype(pc)::value;
        if (e0) {
          StepArgs aa = a;
          const int4* sl = a.slot;
          float2* ob = a.obj;
          int n = a.n;
          void* args[] = {&sl, &ob, &n, &aa};
          return hipExtLaunchKernel((const void*)k_patch_step<M, V, LV, PH>, dim3(a.b), dim3(NT),
                                    args, 0, s, e0, e1, 0);
        }
        hipLaunchKernelGGL((k_patch_step<M, V, LV, PH>), dim3(a.b), dim3(NT), 0, s, a.slot, a.obj,
                           a.n, a);
        return hipGetLastError();
      });
    });
  });
}

template <int M>
hipError_t Launchers<M>::finalize(int f, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                                  hipEvent_t e1) {
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

template <int M>
hipError_t Launchers<M>::patch_step_multi(int v, int L, const StepArgs* args, const int2* work,
                                          int blocks, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    return with_levels(L, [&](auto lc) {
      constexpr int V = decltype(vc)::value, LV = decltype(lc)::value;
      // the records live on the device: the phase memory is tested per instance
      hipLaunchKernelGGL((k_patch_step_multi<M, V, LV, true>), dim3(blocks), dim3(Plan<M, V>::NT),
                         0, s, args, work);
      return hipGetLastError();
    });
  });
}

template <int M>
hipError_t Launchers<M>::finalize_multi(int f, const StepArgs* args, const int2* work, int blocks,
                                        hipStream_t s) {
  return with_fin(f, [&](auto fc) {
    constexpr int F = decltype(fc)::value;
    hipLaunchKernelGGL((k_finalize_multi<M, F>), dim3(blocks), dim3(FinShape<F>::FNT), 0, s, args,
                       work);
    return hipGetLastError();
  });
}

template <int M>
hipError_t Launchers<M>::finalize_item_count(int f, int nr, int nc, int pgroups, int* items) {
  return with_fin(f, [&](auto fc) {
    constexpr int F = decltype(fc)::value;
    int ntiles = 0;
    *items = finalize_items<M, FinShape<F>::FNT, FinShape<F>::T>(nr, nc, pgroups, &ntiles);
    return hipSuccess;
  });
}

template <int M>
hipError_t Launchers<M>::plain_step(int v, int L, const StepArgs& a, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    return with_levels(L, [&](auto lc) {
      constexpr int V = decltype(vc)::value, LV = decltype(lc)::value, NT = Plan<M, V>::NT;
      hipLaunchKernelGGL((k_probe_prep<M, V>), dim3(1), dim3(NT), 0, s, a);
      hipLaunchKernelGGL((k_gather<M, V>), dim3(a.b), dim3(NT), 0, s, a);
      hipLaunchKernelGGL((k_fft<M, V, false>), dim3(a.b), dim3(NT), 0, s, a);
      hipLaunchKernelGGL((k_project<M, V>), dim3(a.b), dim3(NT), 0, s, a);
      hipLaunchKernelGGL((k_fft<M, V, true>), dim3(a.b), dim3(NT), 0, s, a);
      hipLaunchKernelGGL((k_numerators<M, V, LV>), dim3(a.b), dim3(NT), 0, s, a);
      return hipGetLastError();
    });
  });
}

template <int M>
hipError_t Launchers<M>::persistent_grid_size(int v, int L, int num_cus, int* grid) {
  return with_plan<M>(v, [&](auto vc) {
    return with_levels(L, [&](auto lc) {
      constexpr int V = decltype(vc)::value, LV = decltype(lc)::value;
      // the smaller of the two forms' residencies, so either launch fits
      int per0 = 0, per1 = 0;
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per0, k_epoch_persistent<M, V, LV, false>, Plan<M, V>::NT, 0);
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per1, k_epoch_persistent<M, V, LV, true>, Plan<M, V>::NT, 0);
      if (e != hipSuccess) return e;
      *grid = min(per0, per1) * num_cus;
      return hipSuccess;
    });
  });
}

template <int M>
hipError_t Launchers<M>::persistent_epoch(int v, int L, const StepArgs& a, int n_pos, int B,
                                          int grid, unsigned* bar, unsigned bar_base, int* err,
                                          unsigned spin_limit, int* used_grid, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    return with_levels(L, [&](auto lc) {
      constexpr int V = decltype(vc)::value, LV = decltype(lc)::value, NT = Plan<M, V>::NT;
      int ntiles;
      int nitems = finalize_items<M, NT, PersistFin<NT>::T>(a.nr, a.n, a.pgroups, &ntiles);
      StepArgs aa = a;
      int np = n_pos, bb = B;
      unsigned* br = bar;
      unsigned bb0 = bar_base;
      int* er = err;
      unsigned sl = spin_limit;
      const int want = max(min(B, n_pos), nitems);
      const int g = max(1, min(grid, want));
      *used_grid = g;
      void* args[] = {&aa, &np, &bb, &ntiles, &nitems, &br, &bb0, &er, &sl};
      const void* fn = a.phase ? (const void*)k_epoch_persistent<M, V, LV, true>
                               : (const void*)k_epoch_persistent<M, V, LV, false>;
      return hipLaunchCooperativeKernel(fn, dim3(g), dim3(NT), args, 0, s);
    });
  });
}

template <int M>
hipError_t Launchers<M>::layout(int v, const float* d, float* dperm, int n_pos, double* sums,
                                int* bad, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    constexpr int V = decltype(vc)::value;
    hipLaunchKernelGGL((k_layout<M, V>), dim3(n_pos), dim3(256), 0, s, d, dperm, sums, bad);
    return hipGetLastError();
  });
}

template <int M>
hipError_t Launchers<M>::normalize(float2* probe, double dp_avg, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize<M>, dim3(1), dim3(256), 0, s, probe, dp_avg, flag);
  return hipGetLastError();
}

template <int M>
hipError_t Launchers<M>::misfit(int v, const float2* obj, int n, const float2* probe,
                                const float* dperm, const int2* pos, const int4* slot, int count,
                                const float2* tw, double* phi_out, int by_pattern, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    constexpr int V = decltype(vc)::value;
    if constexpr (HalfMisfit<M, V>::value)
      hipLaunchKernelGGL((k_misfit_half<M, V>), dim3(count), dim3(HalfMisfit<M, V>::NT), 0, s, obj, n,
                         probe, dperm,
                         pos, slot, tw, phi_out, by_pattern);
    else
      hipLaunchKernelGGL((k_misfit<M, V>), dim3(count), dim3(Plan<M, V>::NT), 0, s, obj, n, probe,
                         dperm, pos, slot, tw, phi_out, by_pattern);
    return hipGetLastError();
  });
}

template <int M>
hipError_t Launchers<M>::surrogate(int v, const StepArgs& a, double* terms, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    constexpr int V = decltype(vc)::value;
    hipLaunchKernelGGL((k_surrogate<M, V>), dim3(a.b), dim3(Plan<M, V>::NT), 0, s, a, terms);
    return hipGetLastError();
  });
}

template <int M>
hipError_t Launchers<M>::revised_waves(int v, const StepArgs& a, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    constexpr int V = decltype(vc)::value, NT = Plan<M, V>::NT;
    hipLaunchKernelGGL((k_probe_prep<M, V>), dim3(1), dim3(NT), 0, s, a);
    hipLaunchKernelGGL((k_gather<M, V>), dim3(a.b), dim3(NT), 0, s, a);
    hipLaunchKernelGGL((k_fft<M, V, false>), dim3(a.b), dim3(NT), 0, s, a);
    hipLaunchKernelGGL((k_project<M, V>), dim3(a.b), dim3(NT), 0, s, a);
    hipLaunchKernelGGL((k_fft<M, V, true>), dim3(a.b), dim3(NT), 0, s, a);
    return hipGetLastError();
  });
}

template <int M>
hipError_t Launchers<M>::numerators(int v, int L, const StepArgs& a, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    return with_levels(L, [&](auto lc) {
      constexpr int V = decltype(vc)::value, LV = decltype(lc)::value;
      hipLaunchKernelGGL((k_numerators<M, V, LV>), dim3(a.b), dim3(Plan<M, V>::NT), 0, s, a);
      return hipGetLastError();
    });
  });
}

template <int M>
hipError_t Launchers<M>::chain(int v, int L, const StepArgs& a, int n_steps, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    return with_levels(L, [&](auto lc) {
      return with_phase(a, [&](auto pc) {
        constexpr int V = decltype(vc)::value, LV = decltype(lc)::value;
        hipLaunchKernelGGL((k_sweep_chain<M, V, LV, decltype(pc)::value>), dim3(1),
                           dim3(Plan<M, V>::NT), 0, s, a, n_steps);
        return hipGetLastError();
      });
    });
  });
}

template <typename T, int M, int V>
static hipError_t grad_t(const GradArgs& g, hipStream_t s) {
  constexpr int NT = Plan<M, V>::NT;
  const int tiles = grad_tiles(g), blocks = tiles + grad_probe_blocks(M);
  for (int k0 = 0; k0 < g.n_pos; k0 += g.chunk) {
    const int cnt = min(g.chunk, g.n_pos - k0);
    const int first = k0 == 0;
    hipLaunchKernelGGL((k_grad_patch<T, M, V>), dim3(cnt), dim3(NT), 0, s, g, k0);
    hipLaunchKernelGGL((k_grad_reduce<T, M>), dim3(blocks), dim3(256 * kGradZGroups), 0, s, g, k0,
                       cnt, first, tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int M>
hipError_t Launchers<M>::grad(int v, bool f64, const GradArgs& g, hipStream_t s) {
  return with_plan<M>(v, [&](auto vc) {
    constexpr int V = decltype(vc)::value;
    if (f64) {
      if constexpr (M <= 64) return grad_t<double, M, V>(g, s);
      return hipErrorInvalidValue;
    }
    return grad_t<float, M, V>(g, s);
  });
}

}  // namespace emg
