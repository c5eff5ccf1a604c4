/*
 * libemagpie — MI355X (gfx950) implementation of the eMAGPIE stochastic
 * surrogate-minimisation epoch for blind ptychographic phase retrieval
 * (Zhang, Deng, Jiang, Di, "Stochastic Multigrid Method for Blind
 * Ptychographic Phase Retrieval", arXiv 2511.01793).
 *
 * Problem statement (Sec. 2.1): recover a complex object z (n_rows x n_cols) and a
 * complex probe Q (m x m) from far-field intensities d_k = |F(Q . P_k z)|^2
 * measured at N scan positions, where P_k selects the m x m window whose
 * top-left corner is positions[k] and F is the unnormalised 2-D DFT.
 *
 * Conventions shared by every entry point:
 *  - All arrays are row-major.  Complex arrays are interleaved {re, im}
 *    pairs: float pairs (complex64) everywhere except the float64 gradient,
 *    which takes double pairs (complex128).
 *  - Pointers named *_dev are device (HBM) pointers; *_host are host
 *    pointers.  The caller owns every buffer it passes; the library never
 *    allocates device memory: its scratch lives in the caller's workspace.
 *  - `stream` is a hipStream_t passed as void*; all device work is
 *    enqueued on it and is asynchronous unless stated otherwise.
 *  - Every call returns an emagpie_status; argument errors are detected on
 *    the host before anything is enqueued and leave all buffers untouched.
 *    emagpie_last_error(ctx) returns a message for the last failure of a
 *    call on that context (NULL: the last failure on the calling thread).
 *  - Device-side errors (a grid barrier of the persistent epoch that gave up
 *    waiting) are raised by the kernel into host-visible memory and returned
 *    as EMAGPIE_E_HIP by the first call on the context made after the failing
 *    work has completed (synchronise the stream to be sure of seeing it);
 *    that call does nothing else, and the state the failing epoch wrote is
 *    not valid.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Results are deterministic: the same inputs give bitwise-identical
 *    outputs (no floating-point atomics; every sum has a fixed order).
 */
#ifndef EMAGPIE_H
#define EMAGPIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct emagpie_ctx_s* emagpie_ctx;

typedef enum {
  EMAGPIE_OK = 0,
  EMAGPIE_E_ARG = -1,         /* null pointer, bad enum, bad scalar            */
  EMAGPIE_E_SHAPE = -2,       /* unsupported m / n / levels / minibatch        */
  EMAGPIE_E_POSITION = -3,    /* a scan window leaves the object               */
  EMAGPIE_E_DATA = -4,        /* NaN or Inf among the intensities              */
  EMAGPIE_E_DEGENERATE = -5,  /* zero probe (normalisation impossible)         */
  EMAGPIE_E_WORKSPACE = -6,   /* workspace missing, misaligned or too small    */
  EMAGPIE_E_HIP = -7,         /* a HIP runtime call failed                     */
  EMAGPIE_E_UNSUPPORTED = -8  /* valid request the library does not provide    */
} emagpie_status;

/* Execution path of emagpie_epoch (all give bitwise-identical results). */
enum {
  EMAGPIE_PATH_PLAIN = 0,  /* one launch per stage, HBM intermediates          */
  EMAGPIE_PATH_FUSED = 1,  /* fused per-patch kernel + finalize kernel         */
  EMAGPIE_PATH_GRAPH = 2,  /* FUSED launches replayed from a captured hipGraph */
  EMAGPIE_PATH_PERSISTENT = 3, /* one cooperative launch per epoch, grid barriers */
  EMAGPIE_PATH_AUTO = 4, /* chosen at init by timing FUSED and GRAPH epochs (and
                            CHAIN when minibatch = 1); PERSISTENT only on request: a
                            cooperative launch slows the process's later launches   */
  EMAGPIE_PATH_CHAIN = 5 /* minibatch 1 only: one workgroup runs the whole sequential
                            sweep, each step applied in place (the paper's literal order,
                            Sec. 3 footnote: positions updated one after another)     */
};

/* fft_plan / finalize_shape value asking emagpie_init to choose by timing */
enum { EMAGPIE_TUNE = -1 };

enum { EMAGPIE_F32 = 0, EMAGPIE_F64 = 1 };

typedef struct {
  int32_t n_rows;       /* object rows (the object is n_rows x n_cols, row-major)   */
  int32_t n_cols;       /* object columns; m <= n_rows, n_cols <= 65536            */
  int32_t m;            /* probe side: 32, 64, 128 or 256                           */
  int32_t n_pos;        /* number of scan positions N >= 1                          */
  int32_t minibatch;    /* B >= 1 positions per update; B = 1 is the paper's
                           sequential sweep (Sec. 2.2, Sec. 3)                       */
  int32_t levels;       /* multigrid levels L: 1 (single level), 2 or 3 (Sec. 3.2)  */
  float alpha;          /* alpha of u_Q = alpha(||Q||_inf^2 - |Q|^2), >= 0 (Sec. 4)  */
  float alpha_z;        /* alpha_z of u_z; 1 = the ePIE probe step (Sec. 4)          */
  int32_t update_probe; /* 1 blind (object and probe); 0 object only                */
  int32_t joint_step;   /* 1: geometric-mean, phase-aligned joint step of Eq. 6
                           (eMAGPIE); 0: take z+ and Q+ directly, the rPIE update of
                           Eq. 2 (with levels = 1)                                  */
  int32_t path;         /* EMAGPIE_PATH_*                                           */
  uint64_t seed;        /* scan-order generator seed                                */
  int32_t fft_plan;     /* kernel shape of the patch stage: 0 .. count-1 (see
                           emagpie_plan_describe; 0 is the default), or EMAGPIE_TUNE */
  int32_t finalize_shape; /* finalize shape 0..11 (0 default; see emagpie_plan_describe),
                           or EMAGPIE_TUNE                                              */
  const char* tune_cache; /* NULL, or a file of autotuning results (JSON lines) that
                           emagpie_init reads before timing and appends to after  */
  int32_t zero_phase_memory; /* 1: the stateful zero-bin phase rule stated after Eq. 3
                           (a bin where F(Q z_k) = 0 takes the phase pattern k had at its
                           previous visit, 0 at the first); the workspace then holds N m^2
                           unit phasors.  0: theta(0) = 0 always (footnote of Def. 2.1). */
} emagpie_config;

/*
 * Kernel plan of a context.  The FFT plan fixes the radix split m = r1 * r2 of
 * the LDS transforms and the threads per patch; the finalize shape fixes the
 * threads per work item, the object tile side and the order the workgroups take
 * the tiles in (fin_order 0: row-major; 1: contiguous bands of tile rows per
 * XCD; 2: tile rows dealt to the XCDs in turn, row r to XCD r mod 8).  Plans
 * that share (r1, r2) give bitwise-identical results; other splits round the
 * same transform differently (and lay the intensities out in their own
 * order).  Finalize shapes never change results.
 */
typedef struct {
  int32_t fft_plan, r1, r2, threads;
  int32_t finalize_shape, fin_threads, fin_tile, fin_order;
  int32_t path;          /* EMAGPIE_PATH_* in use (never AUTO)                       */
  int32_t tuned;         /* 0 fixed by the config, 1 timed at init, 2 from tune_cache */
  int32_t n_fft_plans;   /* candidates timed (0 if the FFT plan was not timed)      */
  float fft_us[4];       /* median patch-stage kernel time per candidate, us        */
  int32_t n_fin_shapes;  /* candidates timed (0 if the shape was not timed)         */
  float fin_us[12];      /* median finalize kernel time per candidate, us           */
  float path_ms[8];      /* median epoch time per path (index EMAGPIE_PATH_*), ms; -1
                            where not timed (PLAIN is never a candidate)            */
} emagpie_plan;

/* Bytes of device workspace a context with this configuration needs. */
emagpie_status emagpie_workspace_size(const emagpie_config* cfg, size_t* bytes);

/*
 * Create a context.  positions_host: N x 2 int32 (row, col) top-left corners,
 * copied; every window must satisfy 0 <= row <= n_rows - m and 0 <= col <=
 * n_cols - m (Sec. 2.1, binary patch operator).  intensities_dev: N x m x m float32 measured intensities,
 * unshifted (zero frequency at [0, 0]); copied into the workspace, so the
 * caller may free it afterwards.  Negative counts act as zero amplitude
 * (a = sqrt(max(d, 0)), Def. 2.1).  workspace_dev must be 256-byte aligned
 * and at least emagpie_workspace_size() bytes; it stays owned by the caller
 * and must outlive the context.  This call synchronises the stream: it
 * returns EMAGPIE_E_DATA if any intensity is NaN or Inf.
 *
 * Autotuning (fft_plan or finalize_shape = EMAGPIE_TUNE, or path =
 * EMAGPIE_PATH_AUTO): unless tune_cache holds a result for this device and
 * problem shape, init times the candidates on the given intensities and
 * positions with a scratch state held in the workspace: each FFT plan's
 * patch-stage kernel and each finalize shape over minibatches of the epoch-0
 * scan order, then whole epochs of each candidate path (fused and graph, and
 * chain when minibatch = 1); it keeps the fastest and appends
 * it to tune_cache.  The caller's buffers are not touched.  A tune_cache that
 * cannot be read or written is ignored.
 */
emagpie_status emagpie_init(emagpie_ctx* out, const emagpie_config* cfg,
                            const int32_t* positions_host, const float* intensities_dev,
                            void* workspace_dev, size_t workspace_bytes, void* stream);

emagpie_status emagpie_destroy(emagpie_ctx ctx);

/* dp_avg = sqrt(sum_ij mean_k d_k,ij) / m, computed in float64 at init (Sec. 4.1). */
emagpie_status emagpie_dp_avg(emagpie_ctx ctx, double* dp_avg_host);

/*
 * Probe normalisation of Sec. 4.1: probe <- probe * dp_avg / ||probe||_2,
 * in place on an m x m complex64 probe.  Synchronises the stream;
 * EMAGPIE_E_DEGENERATE if the probe is zero.
 */
emagpie_status emagpie_normalize_probe(emagpie_ctx ctx, void* probe_dev, void* stream);

/*
 * One eMAGPIE minibatch update (Sec. 3, Prop. 3.2 joint step, Sec. 3.2
 * multigrid object step), in place on obj_dev (n_rows x n_cols complex64) and
 * probe_dev (m x m complex64).  batch_idx_dev: b int32 scan indices in
 * [0, N) (distinct); all of them see the state at the start of the batch.
 * The object step minimises the summed regularised surrogates of the batch
 * (numerator / denominator accumulation in ascending slot order), the probe
 * step the summed Eq. 8 surrogates; then the geometric-mean, phase-aligned
 * joint step of Eq. 6 is applied once per touched object pixel and per probe
 * pixel.  With b = 1 and levels = 1 this is exactly the paper's Prop. 3.2
 * step.  If sampled_misfit_dev (one double) is not null, sum_k Phi_k at the
 * batch-start state (Eq. 1 terms) is ADDED to it.  1 <= b <= minibatch.
 */
emagpie_status emagpie_step_minibatch(emagpie_ctx ctx, void* obj_dev, void* probe_dev,
                                      const int32_t* batch_idx_dev, int32_t b,
                                      double* sampled_misfit_dev, void* stream);

/*
 * One sweep over all N positions in consecutive minibatches of `minibatch`
 * (the last may be shorter), in the scan order perm_dev (N int32, device) or,
 * if perm_dev is null, in the library's order for (seed, epoch): a
 * Fisher-Yates shuffle driven by SplitMix64 (see emagpie_permutation).  If
 * sampled_misfit_dev is not null it is overwritten with the sum of the
 * sampled misfits of the sweep.  The path in the config selects the launch
 * strategy; results do not depend on it.  In the library's own order each
 * minibatch is listed for the device's XCDs before its slots are summed:
 * sorted by window corner and dealt in one contiguous part per XCD (when the
 * XCD count divides the minibatch and it has at least two slots per XCD), so
 * the rounding order of the sums, and with it the last bits, can differ
 * between devices with different XCD counts.  A caller's perm_dev is used as
 * given.
 */
emagpie_status emagpie_epoch(emagpie_ctx ctx, void* obj_dev, void* probe_dev, int64_t epoch,
                             const int32_t* perm_dev, double* sampled_misfit_dev, void* stream);

/*
 * The MAGPIE object minimiser of Sec. 3.2 (closed forms after Eq. 15) for each
 * patch of the batch, before any accumulation or joint step:
 * zplus_dev[s] = z'_k + conj(Q)(R_k - Q z'_k)/(u + |Q|^2), b x m x m complex64.
 * Inputs are not modified.
 */
emagpie_status emagpie_mg_cycle(emagpie_ctx ctx, const void* obj_dev, const void* probe_dev,
                                const int32_t* batch_idx_dev, int32_t b, void* zplus_dev,
                                void* stream);

/*
 * Descent check of one minibatch update (the quadratic surrogate of Eq. 3 and
 * the sampled objective agreement and majorisation of Prop. 3.1).  Applies the
 * same update as emagpie_step_minibatch to obj_dev / probe_dev (in place; the
 * result is bitwise identical) and writes three float64 values to out3_dev:
 *   [0] Phi_B before the step (= the surrogate there, objective agreement),
 *   [1] surrogate after the step, 1/2 sum_k ||Q' . z'_k - R_k||^2 with the
 *       revised waves R_k frozen at the state before the step,
 *   [2] Phi_B after the step (<= [1] by majorisation).
 * Prop. 3.2 guarantees [1] <= [0] for b = 1 and levels = 1.  Each value is an
 * FP64 sum, in a fixed order, of terms formed from FP32 state.  Uses the
 * plain-path kernels plus two reductions (at m = 256 the row-strip and
 * column-block kernels, with the revised waves kept in the stack buffer); it is
 * meant for checking, not speed.
 */
emagpie_status emagpie_check_step(emagpie_ctx ctx, void* obj_dev, void* probe_dev,
                                  const int32_t* batch_idx_dev, int32_t b, double* out3_dev,
                                  void* stream);

/* Exit-wave misfit Phi(Q, z) of Eq. 1 over all N positions, float64 sum, to misfit_dev. */
emagpie_status emagpie_misfit(emagpie_ctx ctx, const void* obj_dev, const void* probe_dev,
                              double* misfit_dev, void* stream);

/*
 * Gradients of Phi (Sec. 2.1, CR calculus; gradient = d/dx + i d/dy):
 * grad_obj = sum_k P_k^T conj(Q)(Q z_k - R_k) (n_rows x n_cols), grad_probe = sum_k
 * conj(z_k)(Q z_k - R_k) (m x m), and Phi to misfit_dev.  dtype EMAGPIE_F32
 * takes complex64 obj/probe/gradients (every m; at m = 256 the patterns go in
 * chunks of the minibatch through the row-strip and column-block kernels),
 * EMAGPIE_F64 complex128 (m <= 64; EMAGPIE_E_UNSUPPORTED otherwise).  Gradients
 * are overwritten, not accumulated.
 */
emagpie_status emagpie_grad(emagpie_ctx ctx, const void* obj_dev, const void* probe_dev,
                            void* grad_obj_dev, void* grad_probe_dev, double* misfit_dev,
                            int32_t dtype, void* stream);

/*
 * The library's scan order for (seed, epoch): Durstenfeld's Fisher-Yates
 * shuffle of 0..n-1; SplitMix64 starting from seed XOR (epoch *
 * 0x9E3779B97F4A7C15); slot i swaps with floor(x * (i + 1) / 2^64).  Host only.
 */
emagpie_status emagpie_permutation(uint64_t seed, int64_t epoch, int32_t n, int32_t* out_host);

/*
 * Kernel timing for benchmarks.  While enabled, the fused path's patch-stage
 * and finalize kernels are launched with HIP events that the runtime
 * timestamps at the kernel's own start and end; the plain path's six
 * patch-stage kernels and every persistent-epoch launch are bracketed by
 * events recorded on the caller's stream.  Captured-graph replays are not
 * instrumented.  Host only; events are library-owned host objects.
 */
emagpie_status emagpie_profile_enable(emagpie_ctx ctx, int32_t enable);

/*
 * Wait for the recorded events and return, per category (0 patch stage,
 * 1 finalize, 2 persistent epoch), the summed milliseconds (ms3_host) and the
 * number of timed launches (count3_host) since the previous read; then reset.
 */
emagpie_status emagpie_profile_read(emagpie_ctx ctx, double* ms3_host, int64_t* count3_host);

/*
 * Many independent reconstructions advanced together (batched instances).
 * A group binds n_inst existing contexts (each made by emagpie_init with its
 * own configuration, data and workspace; sizes and probe sides may differ).
 * emagpie_group_epoch runs one sweep of every instance: step j processes
 * minibatch j of every instance that has one, with one patch-stage launch
 * and one finalize launch per probe-size class covering all instances, the
 * whole sweep replayed from a captured hipGraph whose probe-size classes run
 * as parallel branches.  Each instance's arithmetic is exactly that of
 * emagpie_epoch on its own context (same scan order for the same epoch), so
 * the results are bitwise identical to running the instances one by one.
 * The group workspace (device, 256-byte aligned, emagpie_group_workspace_size
 * bytes) holds the per-step argument records, work lists and scan orders; it
 * is caller-owned and must outlive the group, as must the contexts.
 */
typedef struct emagpie_group_s* emagpie_group;
emagpie_status emagpie_group_workspace_size(int32_t n_inst, const emagpie_ctx* ctxs, size_t* bytes);
emagpie_status emagpie_group_create(emagpie_group* out, int32_t n_inst, const emagpie_ctx* ctxs,
                                    void* workspace_dev, size_t workspace_bytes, void* stream);
/* obj_devs / probe_devs: n_inst device pointers (host array); sampled_misfit_dev:
   nullable, n_inst doubles overwritten with each instance's sampled misfit */
emagpie_status emagpie_group_epoch(emagpie_group g, void* const* obj_devs, void* const* probe_devs,
                                   int64_t epoch, double* sampled_misfit_dev, void* stream);
emagpie_status emagpie_group_destroy(emagpie_group g);

/*
 * Zero-bin phase memory (zero_phase_memory = 1): set every stored phase back to
 * 0, i.e. the state of a run's first sweep.  EMAGPIE_E_ARG if the context has no
 * phase memory.  Stream-ordered.
 */
emagpie_status emagpie_phase_memory_reset(emagpie_ctx ctx, void* stream);

/*
 * The plan a context runs with (after any autotuning at init).  Host only.
 */
emagpie_status emagpie_plan_get(emagpie_ctx ctx, emagpie_plan* out_host);

/*
 * Describe FFT plan fft_plan and finalize shape finalize_shape for probe side
 * m without a context or a GPU (fills the shape fields of out_host; the
 * timing fields are zero).  EMAGPIE_E_ARG if either does not exist for m;
 * *count_host (nullable) receives the number of FFT plans for m.
 */
emagpie_status emagpie_plan_describe(int32_t m, int32_t fft_plan, int32_t finalize_shape,
                                     emagpie_plan* out_host, int32_t* count_host);

/*
 * Message describing the last failure of a call on ctx (a context of either
 * kind; "" if none), or with ctx = NULL the last failure of any call on the
 * calling thread (including calls that could not take a context: a failed
 * init, workspace sizing, ...).  The string stays valid until the next call
 * that fails on the same context / thread, or until the context is destroyed.
 */
const char* emagpie_last_error(emagpie_ctx ctx);

/*
 * Many independent reconstructions behind one context (batched instances,
 * single-handle form of the group API above).  emagpie_init_many creates n_inst member
 * contexts, each exactly as emagpie_init would from cfgs[i], positions_host[i]
 * and intensities_dev[i] (each autotunes at init if its config asks to), plus a
 * group of them, all inside one caller workspace of emagpie_workspace_size_many
 * bytes (256-byte aligned; it must outlive the context).  emagpie_epoch_many is
 * emagpie_group_epoch over the members: one sweep of every instance, bitwise the
 * result of emagpie_epoch on each member alone.  obj_devs / probe_devs are host
 * arrays of n_inst device pointers; sampled_misfit_dev (nullable) receives n_inst
 * doubles.  emagpie_many_member returns member i (owned by the many-context: do
 * not destroy it) for the per-instance calls (misfit, grad, normalize_probe,
 * step, ...).  emagpie_destroy on the many-context releases members and group.
 * Single-instance calls on the many-context itself return EMAGPIE_E_ARG.
 */
emagpie_status emagpie_workspace_size_many(int32_t n_inst, const emagpie_config* cfgs, size_t* bytes);
emagpie_status emagpie_init_many(emagpie_ctx* out, int32_t n_inst, const emagpie_config* cfgs,
                                 const int32_t* const* positions_host,
                                 const float* const* intensities_dev, void* workspace_dev,
                                 size_t workspace_bytes, void* stream);
emagpie_status emagpie_epoch_many(emagpie_ctx ctx, void* const* obj_devs, void* const* probe_devs,
                                  int64_t epoch, double* sampled_misfit_dev, void* stream);
emagpie_status emagpie_many_member(emagpie_ctx ctx, int32_t i, emagpie_ctx* member_out);

/*
 * Exit-wave misfit Phi(Q, z) of Eq. 1, like emagpie_misfit, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): it needs no context and no workspace, and calls no allocating
 * routine.  Its scratch, the per-pattern terms, is a fixed array of the library's own
 * (at most 65536 patterns: 512 KiB per device, held until the process ends).  Every call
 * on a device shares that device's array, so calls that overlap on one device (several
 * streams) race; calls ordered on one stream do not.
 *   positions_dev: n_pos x 2 int32 (row, col) window corners on the device; they must
 *     satisfy 0 <= row <= n_rows - m, 0 <= col <= n_cols - m (not checked on the host:
 *     the kernel clamps each window into the object, so no access leaves the buffers, and
 *     the value for an invalid window is undefined);
 *   intensities_dev: n_pos x m x m float32 measured intensities, natural (unshifted)
 *     order, read in place;
 *   obj_dev (n_rows x n_cols), probe_dev (m x m): complex64; misfit_dev: one double.
 * m = 32, 64 or 128 (EMAGPIE_E_UNSUPPORTED for 256); 1 <= n_pos <= 65536 (EMAGPIE_E_SHAPE
 * otherwise).  The arithmetic is that of emagpie_misfit with FFT plan 0, so the value is
 * bitwise the one a context with plan 0 returns for the same inputs.  Stream-ordered.
 */
emagpie_status emagpie_misfit_noalloc(int32_t n_rows, int32_t n_cols, int32_t m, int32_t n_pos,
                                      const int32_t* positions_dev, const float* intensities_dev,
                                      const void* obj_dev, const void* probe_dev, double* misfit_dev,
                                      void* stream);

/*
 * Fault-injection hook for the device-side error path of the persistent epoch
 * (tests only).  Later persistent epochs of ctx poll each grid barrier at most
 * spin_limit times (0 restores the default, 2^25) and wait for target_skew more
 * arrivals than the grid makes, so with target_skew > 0 every barrier wait gives
 * up after spin_limit polls: the kernel still runs to its end (its results are
 * then not valid) and raises the device error that the next call returns.
 * Host only.
 */
emagpie_status emagpie_debug_barrier(emagpie_ctx ctx, uint32_t spin_limit, uint32_t target_skew);

/*
 * Measured peaks for the roofline, on the caller's device buffer (bytes >=
 * 4 MiB, 256-byte aligned): out2_host[0] = copy bandwidth in GB/s (a plain
 * 16-byte-per-lane device copy from the first half of the buffer to the second;
 * bytes read plus bytes written over the median kernel time of reps launches),
 * out2_host[1] = FP32 vector rate in TFLOP/s (independent fused multiply-adds,
 * 2 flops each, built like the method's kernels: packed FP32 forms disabled).
 * Overwrites the buffer; synchronises the stream.
 */
emagpie_status emagpie_measure_peaks(void* buf_dev, size_t bytes, int32_t reps, double* out2_host,
                                     void* stream);

/* Library version string. */
const char* emagpie_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EMAGPIE_H */
