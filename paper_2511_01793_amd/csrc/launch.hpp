// Host-side launchers for the eMAGPIE kernels (kernels.hpp, kernels_common.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emg {

constexpr int kMaxSlots = 1024;  // patches per minibatch / gradient chunk

struct StepArgs {
  // state (complex64, interleaved)
  float2* obj;       // nr x n (row-major; n is the row stride)
  int n;             // object columns
  int nr;            // object rows
  float2* probe;     // m x m
  // measured data in transform order, scan windows
  const float* dperm;  // N x m x m
  const int2* pos;     // N (row, col)
  const int4* slot;    // b entries: (scan index k, window row, window col, 0)
  int b;
  float alpha, alpha_z;
  int update_probe;
  int joint;         // 1: Eq. 6 joint step; 0: z <- z+, Q <- Q+ (Eq. 2)
  int pgroups;       // slot groups of the probe sums (probe_groups(minibatch))
  float* part_q;     // m = 256: per (slot, row strip) max |Q|^2 and max |z_k|^2,
  float* part_z;     //   per (slot, column block) partial misfit sums
  double* part_phi;
  float2* phase;     // nullable: N x m^2 unit phasors of the zero-bin phase rule (transform order)
  int phase_write;   // 1: store the phasors used (a step); 0: read only
  const float2* tw;  // m twiddles exp(-2 pi i j / m)
  // per-slot products of the patch stage
  float2* numer;     // b x m^2 object numerators conj(Q) R + u z'
  float2* pnum;      // b x m^2 probe numerators conj(z) R + u_z Q
  float* pden;       // b x m^2 probe denominators |z|^2 + u_z
  float* pden_slot;  // b: when not null (alpha_z = 1) the denominator is max |z_k|^2 per slot
  double* phi;       // b sampled misfit terms
  float* Dbuf;       // m^2 object denominators |Q|^2 + u (written by slot 0)
  double* sampled;   // nullable accumulator of sum phi
  float2* zplus;     // nullable: MAGPIE z+_k per slot (mg_cycle output)
  // plain-path intermediates
  float2* stack;     // b x m^2
  float* zmax;       // b
  float* ubuf;       // m^2
  float* qqmax;      // 1
};

// Kernel plans: v = FFT plan variant, f = finalize shape (plans.hpp).  The
// variant must be the one the intensities were laid out with.

// e0 / e1 (optional): events timestamped at the kernel's start and end
hipError_t launch_patch_step(int m, int v, int L, const StepArgs& a, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_finalize(int m, int f, const StepArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
// Many instances per launch: block b runs work[b] = (record in args, slot) for
// the patch stage, or (record in args, finalize item) for the finalize.
hipError_t launch_patch_step_multi(int m, int v, int L, const StepArgs* args, const int2* work,
                                   int blocks, hipStream_t s);
hipError_t launch_finalize_multi(int m, int f, const StepArgs* args, const int2* work, int blocks,
                                 hipStream_t s);
// number of finalize work items (object tiles + probe units) for an nr x nc object
hipError_t finalize_item_count(int m, int f, int nr, int nc, int pgroups, int* items);

// plain path: the six patch-stage kernels (finalize is launched separately)
hipError_t launch_plain_step(int m, int v, int L, const StepArgs& a, hipStream_t s);

// Persistent epoch: one cooperative launch runs every minibatch of a sweep.
// a.slot must point at the slot list of the whole sweep (N entries); a.b is ignored.
// `bar` is a device counter that only grows: the kernel's barriers wait for
// bar_base + (i + 1) * grid arrivals; `err` (device-visible, possibly host memory) is set
// if a barrier wait gives up after spin_limit polls.
hipError_t persistent_grid_size(int m, int v, int L, int num_cus, int* grid);
hipError_t launch_persistent_epoch(int m, int v, int L, const StepArgs& a, int n_pos, int minibatch,
                                   int grid, unsigned* bar, unsigned bar_base, int* err,
                                   unsigned spin_limit, int* used_grid, hipStream_t s);
// zero 64 consecutive unsigned counters
hipError_t launch_zero_u32(unsigned* p, hipStream_t s);

// slot[j] = (idx[j], pos[idx[j]]) for j < count; indices outside [0, n_pos)
// are clamped so that no access leaves the buffers (the result is then undefined)
hipError_t launch_slot_info(const int* idx, const int2* pos, int n_pos, int4* slot, int count,
                            hipStream_t s);

// zero `count` doubles
hipError_t launch_zero_doubles(double* p, int count, hipStream_t s);
// out[0] = sum_{i < count} in[i] in a fixed order
hipError_t launch_sum_doubles(const double* in, int count, double* out, hipStream_t s);
// p[i] = v for i < count
hipError_t launch_fill_c64(float2* p, size_t count, float2 v, hipStream_t s);

// Copy intensities into the transform order of plan v, flag non-finite
// values, and write per-pattern float64 sums.
hipError_t launch_layout_intensities(int m, int v, const float* d, float* dperm, int n_pos,
                                     double* pattern_sums, int* bad_flag, hipStream_t s);

// probe <- probe * dp_avg / ||probe||; flag when the norm is zero
hipError_t launch_normalize_probe(int m, float2* probe, double dp_avg, int* zero_flag,
                                  hipStream_t s);

// One workgroup runs a whole sequential sweep (minibatch 1): a.slot points at n_steps
// slots; each step's update is applied directly to the object window and the probe.
hipError_t launch_chain_sweep(int m, int v, int L, const StepArgs& a, int n_steps, hipStream_t s);

// misfit terms, unreduced: of all patterns (slot == nullptr; count = N, pattern k at
// pos[k]) or of the count patterns of a slot list -> phi_out (count doubles): term j of
// the list at phi_out[j], or at phi_out[k] (its pattern's index) when by_pattern is set
hipError_t launch_misfit_terms(int m, int v, const float2* obj, int n, const float2* probe,
                               const float* dperm, const int2* pos, const int4* slot, int count,
                               const float2* tw, double* phi_out, int by_pattern, hipStream_t s);

// Check mode of one minibatch, in three parts on a.slot / a.b:
//   revised waves R_k of the current state into a.stack and Phi_k into a.phi (the plain
//   path's first five kernels); numerators from a.stack (its sixth); surrogate terms
//   1/2 ||Q . z_k - R_k||^2 of the current state against a.stack.
hipError_t launch_revised_waves(int m, int v, const StepArgs& a, hipStream_t s);
hipError_t launch_numerators(int m, int v, int L, const StepArgs& a, hipStream_t s);
hipError_t launch_surrogate_terms(int m, int v, const StepArgs& a, double* terms, hipStream_t s);

// gradient of the misfit (float or double state), chunked over patterns
struct GradArgs {
  const void* obj;
  int n;               // object columns (row stride)
  int nr;              // object rows
  const void* probe;
  const float* dperm;
  const int2* pos;
  int n_pos;
  int chunk;           // patterns per chunk (<= kMaxSlots)
  const void* tw;      // twiddles in the gradient precision
  void* gobj;          // nr x n
  void* gprobe;        // m x m
  void* gz_slots;      // chunk x m^2
  void* gq_slots;      // chunk x m^2
  double* phi_all;     // N
};
hipError_t launch_grad(int m, int v, bool f64, const GradArgs& g, hipStream_t s);

// m = 256 misfit terms of patterns k0 .. k0 + count - 1 (count <= the context's
// minibatch; uses a.stack and the part_* buffers) -> phi_out[0 .. count)
// m = 256 gradient: chunks of g.chunk patterns (<= the context's minibatch) through the
// strip and column-block kernels over a.stack and a.part_*, then the shared reductions
hipError_t launch_grad256(const StepArgs& a, const GradArgs& g, hipStream_t s);
// m = 256 descent check of the minibatch a.slot / a.b: the step (revised waves kept in
// a.stack), the finalize, then out3[1] (surrogate) and out3[2] (Phi_B after); out3 zeroed
// by the caller, out3[0] accumulated by the finalize
hipError_t launch_check256(const StepArgs& a, int levels, int finalize_shape, double* out3,
                           hipStream_t s);

hipError_t launch_misfit_strips(int m, const StepArgs& a, int k0, int count, double* phi_out,
                                hipStream_t s);

// Calibration kernels (kernels_peak.hip): a copy of n4 16-byte elements with `blocks`
// workgroups of 256 threads, and a loop of independent FP32 FMAs (iters rounds of 16 per
// lane; *flops receives the flop count of the launch).
hipError_t launch_copy16(const void* src, void* dst, size_t n4, int blocks, hipStream_t s);
hipError_t launch_fma_loop(float* out, int blocks, int iters, hipStream_t s, double* flops);

// The launchers of one probe side (kernels.hpp; instantiated per side in
// kernels_m32.hip, kernels_m64.hip and kernels_m128.hip).
template <int M>
struct Launchers {
  static hipError_t patch_step(int v, int L, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1);
  static hipError_t finalize(int f, const StepArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  static hipError_t patch_step_multi(int v, int L, const StepArgs* args, const int2* work,
                                     int blocks, hipStream_t s);
  static hipError_t finalize_multi(int f, const StepArgs* args, const int2* work, int blocks,
                                   hipStream_t s);
  static hipError_t finalize_item_count(int f, int nr, int nc, int pgroups, int* items);
  static hipError_t plain_step(int v, int L, const StepArgs& a, hipStream_t s);
  static hipError_t persistent_grid_size(int v, int L, int num_cus, int* grid);
  static hipError_t persistent_epoch(int v, int L, const StepArgs& a, int n_pos, int B, int grid,
                                     unsigned* bar, unsigned bar_base, int* err,
                                     unsigned spin_limit, int* used_grid, hipStream_t s);
  static hipError_t layout(int v, const float* d, float* dperm, int n_pos, double* sums, int* bad,
                           hipStream_t s);
  static hipError_t normalize(float2* probe, double dp_avg, int* flag, hipStream_t s);
  static hipError_t misfit(int v, const float2* obj, int n, const float2* probe, const float* dperm,
                           const int2* pos, const int4* slot, int count, const float2* tw,
                           double* phi_out, int by_pattern, hipStream_t s);
  static hipError_t revised_waves(int v, const StepArgs& a, hipStream_t s);
  static hipError_t numerators(int v, int L, const StepArgs& a, hipStream_t s);
  static hipError_t surrogate(int v, const StepArgs& a, double* terms, hipStream_t s);
  static hipError_t grad(int v, bool f64, const GradArgs& g, hipStream_t s);
  static hipError_t chain(int v, int L, const StepArgs& a, int n_steps, hipStream_t s);
};

// m = 256 (kernels_m256.hip): the same members; the tile exceeds
// LDS, so a patch runs as row strips and column blocks over a.stack.  Members with
// no m = 256 form return hipErrorInvalidValue (the host rejects those requests
// before launching).
struct Launchers256 {
  static hipError_t patch_step(int v, int L, const StepArgs& a, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1);
  static hipError_t finalize(int f, const StepArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
  static hipError_t patch_step_multi(int v, int L, const StepArgs* args, const int2* work,
                                     int blocks, hipStream_t s);
  static hipError_t finalize_multi(int f, const StepArgs* args, const int2* work, int blocks,
                                   hipStream_t s);
  static hipError_t finalize_item_count(int f, int nr, int nc, int pgroups, int* items);
  static hipError_t plain_step(int v, int L, const StepArgs& a, hipStream_t s);
  static hipError_t persistent_grid_size(int v, int L, int num_cus, int* grid);
  static hipError_t persistent_epoch(int v, int L, const StepArgs& a, int n_pos, int B, int grid,
                                     unsigned* bar, unsigned bar_base, int* err,
                                     unsigned spin_limit, int* used_grid, hipStream_t s);
  static hipError_t layout(int v, const float* d, float* dperm, int n_pos, double* sums, int* bad,
                           hipStream_t s);
  static hipError_t normalize(float2* probe, double dp_avg, int* flag, hipStream_t s);
  static hipError_t misfit(int v, const float2* obj, int n, const float2* probe, const float* dperm,
                           const int2* pos, const int4* slot, int count, const float2* tw,
                           double* phi_out, int by_pattern, hipStream_t s);
  static hipError_t revised_waves(int v, const StepArgs& a, hipStream_t s);
  static hipError_t numerators(int v, int L, const StepArgs& a, hipStream_t s);
  static hipError_t surrogate(int v, const StepArgs& a, double* terms, hipStream_t s);
  static hipError_t grad(int v, bool f64, const GradArgs& g, hipStream_t s);
  static hipError_t chain(int v, int L, const StepArgs& a, int n_steps, hipStream_t s);
  static hipError_t misfit_strips(const StepArgs& a, int k0, int count, double* phi_out,
                                  hipStream_t s);
};

}  // namespace emg
