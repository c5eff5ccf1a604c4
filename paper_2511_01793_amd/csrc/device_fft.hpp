// LDS-resident 2-D FFT for one m x m complex tile per workgroup (gfx950).
//
// The transform is the unnormalised DFT of Sec. 2.1.  Each 1-D length-m
// transform is a two-pass Cooley-Tukey factorisation m = R1 * R2 computed in
// place in LDS: pass 1 does R2-point DFTs over stride-R1 elements and applies
// the twiddles W_m^(n1 k2); pass 2 does R1-point DFTs over contiguous runs.
// Both passes write back to the locations they read, so each pass needs one
// barrier.  The forward transform therefore leaves the spectrum in
// "transform order": LDS position p holds frequency p / R1 + R2 * (p % R1)
// along each axis.  The inverse passes are the conjugate transposes in
// reverse order, so they take transform order in and give natural order out.
// Per-pixel work between the two transforms (the modulus projection) reads
// its amplitudes in the same transform order, laid out once at init.
//
// The factorisation and the threads per tile are a plan (plans.hpp).
// LDS rows are padded by one element (row stride m + 1) so that the
// line-parallel thread mapping used for both row and column passes is free
// of bank conflicts.  Twiddles W_m^j = exp(-2 pi i j / m), j < m, come from a
// table built on the host in double precision and staged in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plans.hpp"

namespace emg {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return cx<T>{a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return cx<T>{a.re - b.re, a.im - b.im}; }
// Products use explicit fused multiply-adds (one product rounded, then fused
// into the other).  Floating-point contraction is otherwise off, so each of
// these rounds the same way in every kernel that inlines it.
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
  return cx<T>{fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ cx<T> mul_fma(cx<T> a, cx<T> b) { return mul(a, b); }
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return cx<T>{fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re))};
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return cx<T>{a.re * s, a.im * s}; }
// a + s * b
template <typename T>
__device__ __forceinline__ cx<T> axpy(T s, cx<T> b, cx<T> a) {
  return cx<T>{fma(s, b.re, a.re), fma(s, b.im, a.im)};
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return fma(a.re, a.re, a.im * a.im); }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return cx<T>{a.re, -a.im}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

template <int M>
__host__ __device__ constexpr int lds_stride() { return M + 1; }

// frequency held at LDS position p after a forward pass pair of plan (M, V)
template <int M, int V>
__host__ __device__ __forceinline__ int freq_of_pos(int p) {
  return p / Plan<M, V>::R1 + Plan<M, V>::R2 * (p % Plan<M, V>::R1);
}

// ---------------------------------------------------------------------------
// small DFTs in registers, forward sign exp(-2 pi i jk/R), inverse exp(+...)
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a;
  a = add(t, b);
  b = sub(t, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> y0 = add(a0, a2), y1 = sub(a0, a2), y2 = add(a1, a3), y3 = rot90<T, INV>(sub(a1, a3));
  a0 = add(y0, y2);
  a2 = sub(y0, y2);
  a1 = add(y1, y3);
  a3 = sub(y1, y3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
  // even / odd split: X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  const T h = T(0.70710678118654752440084436210484903928);
  // W8^1 = (h, -h) forward, (h, +h) inverse
  cx<T> t1 = INV ? cx<T>{h * (o1.re - o1.im), h * (o1.re + o1.im)}
                 : cx<T>{h * (o1.re + o1.im), h * (o1.im - o1.re)};
  cx<T> t2 = rot90<T, INV>(o2);
  // W8^3 = (-h, -h) forward, (-h, +h) inverse
  cx<T> t3 = INV ? cx<T>{-h * (o3.re + o3.im), h * (o3.re - o3.im)}
                 : cx<T>{h * (o3.im - o3.re), -h * (o3.re + o3.im)};
  v[0] = add(e0, o0);
  v[4] = sub(e0, o0);
  v[1] = add(e1, t1);
  v[5] = sub(e1, t1);
  v[2] = add(e2, t2);
  v[6] = sub(e2, t2);
  v[3] = add(e3, t3);
  v[7] = sub(e3, t3);
}

// 16-point DFT as two 8-point halves: X_k = E_k + W16^k O_k, X_{k+8} = E_k - W16^k O_k,
// with W16^k = exp(-+2 pi i k / 16) as constants (W16^4 = -+i, W16^2 and W16^6 through
// the 1/sqrt(2) form of the 8-point transform, the odd powers through fused products).
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cx<T>* v) {
  cx<T> e[8], o[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    e[j] = v[2 * j];
    o[j] = v[2 * j + 1];
  }
  dft8<T, INV>(e);
  dft8<T, INV>(o);
  const T c1 = T(0.92387953251128675612818318939678828682);  // cos(pi / 8)
  const T s1 = T(0.38268343236508977172845998403039886676);  // sin(pi / 8)
  const T h = T(0.70710678118654752440084436210484903928);
  const T sg = INV ? T(1) : T(-1);  // sign of the imaginary parts of W16^k, k = 1..7
  cx<T> t[8];
  t[0] = o[0];
  t[1] = mul(cx<T>{c1, sg * s1}, o[1]);
  t[2] = INV ? cx<T>{h * (o[2].re - o[2].im), h * (o[2].re + o[2].im)}
             : cx<T>{h * (o[2].re + o[2].im), h * (o[2].im - o[2].re)};
  t[3] = mul(cx<T>{s1, sg * c1}, o[3]);
  t[4] = rot90<T, INV>(o[4]);
  t[5] = mul(cx<T>{-s1, sg * c1}, o[5]);
  t[6] = INV ? cx<T>{-h * (o[6].re + o[6].im), h * (o[6].re - o[6].im)}
             : cx<T>{h * (o[6].im - o[6].re), -h * (o[6].re + o[6].im)};
  t[7] = mul(cx<T>{-c1, sg * s1}, o[7]);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = add(e[k], t[k]);
    v[k + 8] = sub(e[k], t[k]);
  }
}

template <typename T, bool INV, int R, int M>
__device__ __forceinline__ void dft_small(cx<T>* v, const cx<T>* tw) {
  if constexpr (R == 2) {
    dft2<T, INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<T, INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    dft8<T, INV>(v);
  } else {
    static_assert(R == 16, "radix");
    dft16<T, INV>(v);
  }
}

// ---------------------------------------------------------------------------
// one in-place pass along rows (COLS = false) or columns (COLS = true)
//   STRIDED: DFT over positions g + R1 * j (j < R2), group g = n1 < R1
//   else   : DFT over positions R1 * g + j (j < R1), group g = k2 < R2
//   forward strided pass multiplies output j by W^(g j) after the DFT;
//   inverse strided pass multiplies input j by conj(W^(g j)) before it.
// Work item w -> line = w % M (line fastest: conflict-free with stride M+1).
// ---------------------------------------------------------------------------
template <typename T, int M, int V, bool INV, bool STRIDED, bool COLS>
__device__ __forceinline__ void fft_pass(cx<T>* A, const cx<T>* tw, int tid) {
  constexpr int R1 = Plan<M, V>::R1, R2 = Plan<M, V>::R2, NT = Plan<M, V>::NT;
  constexpr int R = STRIDED ? R2 : R1;
  constexpr int G = STRIDED ? R1 : R2;
  constexpr int ITEMS = M * G;
  constexpr int LS = lds_stride<M>();
  static_assert(ITEMS % NT == 0 || NT % ITEMS == 0, "items per thread");
  constexpr int IT = ITEMS >= NT ? ITEMS / NT : 1;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * NT;
    if (ITEMS < NT && w >= ITEMS) break;
    const int line = w % M;
    const int g = w / M;
    cx<T> v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int p = STRIDED ? (g + R1 * j) : (R1 * g + j);
      const int addr = COLS ? (p * LS + line) : (line * LS + p);
      v[j] = A[addr];
    }
    if (STRIDED && INV) {
#pragma unroll
      for (int j = 1; j < R; ++j) v[j] = mul_fma(conjg(tw[g * j]), v[j]);
    }
    dft_small<T, INV, R, M>(v, tw);
    if (STRIDED && !INV) {
#pragma unroll
      for (int j = 1; j < R; ++j) v[j] = mul_fma(tw[g * j], v[j]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int p = STRIDED ? (g + R1 * j) : (R1 * g + j);
      const int addr = COLS ? (p * LS + line) : (line * LS + p);
      A[addr] = v[j];
    }
  }
}

// Forward 2-D DFT: natural order in, transform order out.  Caller must have
// synchronised after filling A; returns after a final barrier.
template <typename T, int M, int V>
__device__ __forceinline__ void fft2_forward(cx<T>* A, const cx<T>* tw, int tid) {
  fft_pass<T, M, V, false, true, false>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, false, false, false>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, false, true, true>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, false, false, true>(A, tw, tid);
  __syncthreads();
}

// The inverse transform without its first pass.  The last forward pass and the
// first inverse pass are the same contiguous column pass (same items per thread,
// no twiddles), so a caller runs the forward transform's first three passes, then
// both of these in registers with per-element work between them (fft_pass_pair),
// then this tail.
template <typename T, int M, int V>
__device__ __forceinline__ void fft2_inverse_tail(cx<T>* A, const cx<T>* tw, int tid) {
  fft_pass<T, M, V, true, true, true>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, true, false, false>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, true, true, false>(A, tw, tid);
  __syncthreads();
}

// Items of the contiguous column pass: ITEMS = M * R2 lines of R1 points;
// item w covers LDS positions (R1 * (w / M) + j) * (M + 1) + w % M, j < R1.
template <int M, int V>
struct ColPass {
  static constexpr int R1 = Plan<M, V>::R1, R2 = Plan<M, V>::R2, NT = Plan<M, V>::NT;
  static constexpr int ITEMS = M * R2;
  static constexpr int IT = ITEMS >= NT ? ITEMS / NT : 1;  // items per thread
  static constexpr int PTS = IT * R1;                        // points per thread
};

// Last forward pass, f(item point, value) on each transformed value, first
// inverse pass: in registers, one LDS read and one write per point.  Caller
// synchronises before (the head's barrier) and after.
// Last forward pass in registers: each transformed value goes to f(item point,
// value) and is not written back (for consumers that only reduce it).
template <typename T, int M, int V, class F>
__device__ __forceinline__ void fft_pass_last(const cx<T>* A, int tid, F f) {
  using C = ColPass<M, V>;
  constexpr int LS = lds_stride<M>();
#pragma unroll
  for (int it = 0; it < C::IT; ++it) {
    const int w = tid + it * C::NT;
    if (C::ITEMS < C::NT && w >= C::ITEMS) break;
    const int line = w % M, g = w / M;
    cx<T> v[C::R1];
#pragma unroll
    for (int j = 0; j < C::R1; ++j) v[j] = A[(C::R1 * g + j) * LS + line];
    dft_small<T, false, C::R1, M>(v, nullptr);
#pragma unroll
    for (int j = 0; j < C::R1; ++j) f(it * C::R1 + j, v[j]);
  }
}

template <typename T, int M, int V, class F>
__device__ __forceinline__ void fft_pass_pair(cx<T>* A, int tid, F f) {
  using C = ColPass<M, V>;
  constexpr int LS = lds_stride<M>();
#pragma unroll
  for (int it = 0; it < C::IT; ++it) {
    const int w = tid + it * C::NT;
    if (C::ITEMS < C::NT && w >= C::ITEMS) break;
    const int line = w % M, g = w / M;
    cx<T> v[C::R1];
#pragma unroll
    for (int j = 0; j < C::R1; ++j) v[j] = A[(C::R1 * g + j) * LS + line];
    dft_small<T, false, C::R1, M>(v, nullptr);
#pragma unroll
    for (int j = 0; j < C::R1; ++j) f(it * C::R1 + j, v[j]);
    dft_small<T, true, C::R1, M>(v, nullptr);
#pragma unroll
    for (int j = 0; j < C::R1; ++j) A[(C::R1 * g + j) * LS + line] = v[j];
  }
}

// ---------------------------------------------------------------------------
// Register-resident passes for the split m = 8 * 8 with cross-lane transposes.
// A line of 64 points (a row or a column of the tile) lives in the 8 lanes
// base + 8 i (i = 0..7) of one wave, 8 points per lane.  For a strided pass lane
// i holds points i + 8 j in register j: the pass's 8-point DFT and its twiddles
// W^(i j) are lane-local.  An 8 x 8 transpose across the 8 lanes (lane bits
// 3..5 exchanged with register bits 0..2) then leaves lane i holding points
// 8 i + j, the run of the contiguous pass.  The DFTs, the twiddle products and
// their operand order are those of fft_pass, so a tile transformed this way is
// bitwise the tile the LDS passes of the same split give.
// ---------------------------------------------------------------------------
// Exchange between lanes l and l ^ D of a register pair (a, b): lanes with the
// D bit clear take the partner's a into b, lanes with it set take the partner's
// b into a.  D = 8: two DPP moves (row rotation by 8 within 16-lane rows, the
// bank mask picking the receiving half); D = 16, 32: one lane-swap instruction.
// DPP controls: rotate right by 8 lanes within each 16-lane row (lane l reads
// lane l ^ 8), all four rows enabled, and the bank masks (banks are 4-lane
// groups of a row) of its lower and upper 8 lanes
constexpr int kDppRowRor8 = 0x128, kDppAllRows = 0xF, kDppBanksLow8 = 0x3, kDppBanksHigh8 = 0xC;

template <int D>
__device__ __forceinline__ void xl_exchange(float& a, float& b) {
  const int ia = __float_as_int(a), ib = __float_as_int(b);
  if constexpr (D == 8) {
    const int nb =
        __builtin_amdgcn_update_dpp(ib, ia, kDppRowRor8, kDppAllRows, kDppBanksLow8, false);
    const int na =
        __builtin_amdgcn_update_dpp(ia, ib, kDppRowRor8, kDppAllRows, kDppBanksHigh8, false);
    a = __int_as_float(na);
    b = __int_as_float(nb);
  } else if constexpr (D == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)ia, (unsigned)ib, false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
  } else {
    static_assert(D == 32, "lane distance");
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)ia, (unsigned)ib, false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
  }
}

template <int D>
__device__ __forceinline__ void xl_exchange(cx<float>& a, cx<float>& b) {
  xl_exchange<D>(a.re, b.re);
  xl_exchange<D>(a.im, b.im);
}

// v[j] of lane i  ->  v[i] of lane j, for the 8 lanes base + 8 i
__device__ __forceinline__ void xl_transpose8(cx<float>* v) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (!(k & 1)) xl_exchange<8>(v[k], v[k | 1]);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (!(k & 2)) xl_exchange<16>(v[k], v[k | 2]);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (!(k & 4)) xl_exchange<32>(v[k], v[k | 4]);
}

// strided pass of lane i over its points i + 8 j; w[j] = W_64^(i j), j = 1..7
template <bool INV>
__device__ __forceinline__ void xl_strided(cx<float>* v, const cx<float>* w) {
  if constexpr (INV) {
#pragma unroll
    for (int j = 1; j < 8; ++j) v[j] = mul_fma(conjg(w[j]), v[j]);
  }
  dft8<float, INV>(v);
  if constexpr (!INV) {
#pragma unroll
    for (int j = 1; j < 8; ++j) v[j] = mul_fma(w[j], v[j]);
  }
}

// LDS slot of tile element (r, c), 64 x 64 tile: unpadded rows, the column
// XOR-swizzled by 9 (r mod 8).  A wave's 8-lane-group accesses of the row phase
// (rows 8 w .. 8 w + 7, columns 8 i + j or i + 8 j) and of the column phase
// (columns 8 w .. 8 w + 7, rows i + 8 j) then fall in distinct banks.
__device__ __forceinline__ int xl_addr(int r, int c) { return r * 64 + (c ^ (9 * (r & 7))); }

// The LDS passes of fft_pass over a block of LINES independent length-N lines (a
// strip of rows or a block of columns of a tile too large for one workgroup's LDS).
// COLS = false: line l holds A[l * LS + p]; COLS = true: A[p * LS + l].
template <typename T, int N, int R1, int R2, int LINES, int NT, int LS, bool INV, bool STRIDED,
          bool COLS>
__device__ __forceinline__ void fft_pass_lines(cx<T>* A, const cx<T>* tw, int tid) {
  constexpr int R = STRIDED ? R2 : R1;
  constexpr int G = STRIDED ? R1 : R2;
  constexpr int ITEMS = LINES * G;
  static_assert(R1 * R2 == N, "radix split");
  static_assert(ITEMS % NT == 0 || NT % ITEMS == 0, "items per thread");
  constexpr int IT = ITEMS >= NT ? ITEMS / NT : 1;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * NT;
    if (ITEMS < NT && w >= ITEMS) break;
    const int line = w % LINES;
    const int g = w / LINES;
    cx<T> v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int p = STRIDED ? (g + R1 * j) : (R1 * g + j);
      v[j] = A[COLS ? (p * LS + line) : (line * LS + p)];
    }
    if (STRIDED && INV) {
#pragma unroll
      for (int j = 1; j < R; ++j) v[j] = mul_fma(conjg(tw[g * j]), v[j]);
    }
    dft_small<T, INV, R, N>(v, tw);
    if (STRIDED && !INV) {
#pragma unroll
      for (int j = 1; j < R; ++j) v[j] = mul_fma(tw[g * j], v[j]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int p = STRIDED ? (g + R1 * j) : (R1 * g + j);
      A[COLS ? (p * LS + line) : (line * LS + p)] = v[j];
    }
  }
}

// Contiguous pass forward, f(point, value) on each transformed value, contiguous
// pass inverse, in registers (the block form of fft_pass_pair; same items).
// Point e of a thread is item it = e / R1, j = e % R1 at line (tid + it NT) % LINES,
// position R1 ((tid + it NT) / LINES) + j.
template <typename T, int N, int R1, int R2, int LINES, int NT, int LS, bool COLS, class F>
__device__ __forceinline__ void fft_pass_lines_pair(cx<T>* A, int tid, F f) {
  constexpr int ITEMS = LINES * R2;
  constexpr int IT = ITEMS >= NT ? ITEMS / NT : 1;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int w = tid + it * NT;
    if (ITEMS < NT && w >= ITEMS) break;
    const int line = w % LINES, g = w / LINES;
    cx<T> v[R1];
#pragma unroll
    for (int j = 0; j < R1; ++j) {
      const int p = R1 * g + j;
      v[j] = A[COLS ? (p * LS + line) : (line * LS + p)];
    }
    dft_small<T, false, R1, N>(v, nullptr);
#pragma unroll
    for (int j = 0; j < R1; ++j) f(it * R1 + j, v[j]);
    dft_small<T, true, R1, N>(v, nullptr);
#pragma unroll
    for (int j = 0; j < R1; ++j) {
      const int p = R1 * g + j;
      A[COLS ? (p * LS + line) : (line * LS + p)] = v[j];
    }
  }
}

// Inverse 2-D DFT without the 1/m^2 factor: transform order in, natural out.
template <typename T, int M, int V>
__device__ __forceinline__ void fft2_inverse(cx<T>* A, const cx<T>* tw, int tid) {
  fft_pass<T, M, V, true, false, true>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, true, true, true>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, true, false, false>(A, tw, tid);
  __syncthreads();
  fft_pass<T, M, V, true, true, false>(A, tw, tid);
  __syncthreads();
}

// Principal complex square root (W. Kahan, "Branch Cuts for Complex
// Elementary Functions", 1987: t = sqrt((|x| + |w|)/2), the other part from
// y / (2t)), then the sign chosen so Re(root * conj(ref)) >= 0 (Eq. 6).  The
// square roots and the reciprocal are the hardware's (within one ulp each).  A
// product of modulus below 2^-125 (whose root is below 1.5e-19) gives 0; past that
// test the second root and the reciprocal always take normal inputs.
__device__ __forceinline__ cx<float> aligned_sqrt(cx<float> ref, cx<float> plus) {
  const cx<float> w = mul(ref, plus);
  const float mag = __builtin_amdgcn_sqrtf(w.re * w.re + w.im * w.im);
  if (mag < 2.35098870e-38f) return cx<float>{0.f, 0.f};
  const float t = __builtin_amdgcn_sqrtf((fabsf(w.re) + mag) * 0.5f);
  const float h = 0.5f * __builtin_amdgcn_rcpf(t);  // 1 / (2 t)
  cx<float> s = w.re >= 0.f ? cx<float>{t, w.im * h} : cx<float>{fabsf(w.im) * h, copysignf(t, w.im)};
  if (s.re * ref.re + s.im * ref.im < 0.f) s = cx<float>{-s.re, -s.im};
  return s;
}

}  // namespace emg
