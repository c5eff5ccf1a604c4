// libemagpie C ABI: validation, workspace carving, scan order, launch
// strategies (plain, fused, captured hipGraph, persistent cooperative).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "emagpie.h"
#include "launch.hpp"
#include "plans.hpp"

namespace {

// The last failure on this thread, and a count of failures so far: an entry point
// that takes a context copies a failure raised during the call into the context.
thread_local std::string g_err;
thread_local uint64_t g_err_count = 0;

emagpie_status fail(emagpie_status st, const std::string& msg) {
  g_err = msg;
  ++g_err_count;
  return st;
}

}  // namespace

namespace emg {
// failure message of a call made outside this file (the no-allocation misfit)
emagpie_status set_error(emagpie_status st, const std::string& msg) { return fail(st, msg); }
}  // namespace emg

namespace {

#define EMG_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(EMAGPIE_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// SplitMix64 (Steele, Lea, Flood 2014; Vigna's reference definition)
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += kGamma;
    uint64_t x = s;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
  }
};

void fisher_yates(uint64_t seed, int64_t epoch, int32_t n, int32_t* out) {
  SplitMix64 g{seed ^ ((uint64_t)epoch * kGamma)};
  for (int32_t i = 0; i < n; ++i) out[i] = i;
  for (int32_t i = n - 1; i > 0; --i) {
    const uint64_t x = g.next();
    const int32_t j = (int32_t)(((unsigned __int128)x * (uint64_t)(i + 1)) >> 64);
    const int32_t t = out[i];
    out[i] = out[j];
    out[j] = t;
  }
}

// Listing order of one minibatch's slots for the launch.  Workgroup i of a launch
// runs on XCD i mod X (X accelerator complex dies, each with its own L2), so the
// slots are sorted by window corner (row, then column) and the sorted run is dealt
// in X contiguous parts: part x goes to slots x, x + X, x + 2X, ...  Neighbouring
// windows then share an L2 and re-read each other's object pixels from it.  The
// minibatch is a set (every sum over it runs in listing order, the same on every
// launch strategy), so this changes rounding order only.  Left as it is unless
// X > 1 divides b and b >= 2X.
void xcd_listing(int4* d, int b, int xcc, std::vector<int4>& tmp) {
  if (xcc <= 1 || b < 2 * xcc || b % xcc != 0) return;
  tmp.assign(d, d + b);
  std::stable_sort(tmp.begin(), tmp.end(), [](const int4& p, const int4& q) {
    return p.y != q.y ? p.y < q.y : p.z < q.z;
  });
  const int per = b / xcc;
  for (int x = 0; x < xcc; ++x)
    for (int k = 0; k < per; ++k) d[x + xcc * k] = tmp[x * per + k];
}
void xcd_listing_sweep(int4* d, int n, int B, int xcc, std::vector<int4>& tmp) {
  for (int s0 = 0; s0 < n; s0 += B) xcd_listing(d + s0, std::min(B, n - s0), xcc, tmp);
}

// Launch order of the full misfit: every pattern once, sorted by window corner and
// dealt to the XCDs like a minibatch listing (the x-th contiguous part of the sorted
// run to blocks x, x + X, ...), so the windows one XCD transforms lie in one band of
// the object and are re-read from its L2.  When X does not divide n, the last n mod X
// sorted patterns follow at the end.  The terms are stored by pattern index, so the
// order changes no result.
void misfit_order(const int32_t* pos, int n, int xcc, std::vector<int4>& out) {
  std::vector<int4> t(n);
  for (int k = 0; k < n; ++k) t[k] = make_int4(k, pos[2 * k], pos[2 * k + 1], 0);
  std::stable_sort(t.begin(), t.end(), [](const int4& p, const int4& q) {
    return p.y != q.y ? p.y < q.y : p.z < q.z;
  });
  out.resize(n);
  const int X = std::max(1, xcc), per = n / X, head = per * X;
  for (int i = 0; i < head; ++i) out[i] = t[(i % X) * per + i / X];
  for (int i = head; i < n; ++i) out[i] = t[i];
}

struct Region {
  size_t off, bytes;
};

constexpr unsigned kDefaultSpinLimit = 1u << 25;

bool wants_tuning(const emagpie_config& c) {
  return c.fft_plan == EMAGPIE_TUNE || c.finalize_shape == EMAGPIE_TUNE || c.path == EMAGPIE_PATH_AUTO;
}

struct Layout {
  Region dperm, pos, slots, morder, tw32, tw64, numer, pnum, pden, pden_slot, phi, stack, zmax, ubuf, Dbuf,
      scal, bar, phi_all, gz, gq, tune_obj, tune_probe, phase, part;
  int grad_chunk;
  size_t total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const emagpie_config& c) {
  Layout L{};
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    Region r{cur, bytes};
    cur += align256(bytes);
    return r;
  };
  const size_t m2 = (size_t)c.m * c.m, N = (size_t)c.n_pos, B = (size_t)c.minibatch;
  L.dperm = take(N * m2 * 4);
  L.pos = take(N * 8);
  L.slots = take(std::max(N, B) * 16);
  L.morder = take(c.m == 256 ? 0 : N * 16);
  L.tw32 = take((size_t)c.m * 8);
  L.tw64 = take((size_t)c.m * 16);
  L.numer = take(B * m2 * 8);
  L.pnum = take(B * m2 * 8);
  L.pden = take(B * m2 * 4);
  L.pden_slot = take(B * 4);
  L.phi = take(B * 8);
  L.stack = take(B * m2 * 8);
  L.zmax = take(B * 4);
  L.ubuf = take(m2 * 4);
  L.Dbuf = take(m2 * 4);
  L.scal = take(256);
  L.bar = take(256);
  L.phi_all = take(N * 8);
  // patterns per gradient chunk: at m = 256 the stack buffer's minibatch
  L.grad_chunk = (int)std::min<size_t>(N, c.m == 256 ? B : c.m == 128 ? 256 : emg::kMaxSlots);
  const size_t gel = c.m <= 64 ? 16 : 8;  // complex128 where the float64 gradient exists
  L.gz = take((size_t)L.grad_chunk * m2 * gel);
  L.gq = take((size_t)L.grad_chunk * m2 * gel);
  // scratch state for autotuning at init (only when asked for)
  const bool tune = wants_tuning(c);
  L.tune_obj = take(tune ? (size_t)c.n_rows * c.n_cols * 8 : 0);
  L.tune_probe = take(tune ? m2 * 8 : 0);
  L.phase = take(c.zero_phase_memory ? N * m2 * 8 : 0);
  // m = 256: strip maxima and column-block partial misfits per slot (16 of each)
  L.part = take(c.m == 256 ? B * 16 * (4 + 4 + 8) : 0);
  L.total = cur;
  return L;
}

emagpie_status check_config(const emagpie_config* c) {
  if (!c) return fail(EMAGPIE_E_ARG, "null config");
  if (c->m != 32 && c->m != 64 && c->m != 128 && c->m != 256)
    return fail(EMAGPIE_E_SHAPE, "probe side m must be 32, 64, 128 or 256");
  if (c->n_rows < c->m || c->n_rows > 65536 || c->n_cols < c->m || c->n_cols > 65536)
    return fail(EMAGPIE_E_SHAPE, "object sides must satisfy m <= n_rows, n_cols <= 65536");
  if ((size_t)c->n_rows * (size_t)c->n_cols > (size_t)1 << 31)
    return fail(EMAGPIE_E_SHAPE, "object larger than 2^31 pixels");
  if (c->n_pos < 1) return fail(EMAGPIE_E_SHAPE, "n_pos must be >= 1");
  if (c->minibatch < 1 || c->minibatch > emg::kMaxSlots)
    return fail(EMAGPIE_E_SHAPE, "minibatch must be in [1, 1024]");
  if (c->levels < 1 || c->levels > 3) return fail(EMAGPIE_E_SHAPE, "levels must be 1, 2 or 3");
  if (!(c->alpha >= 0.f) || !std::isfinite(c->alpha)) return fail(EMAGPIE_E_ARG, "alpha must be finite and >= 0");
  if (!(c->alpha_z >= 0.f) || !std::isfinite(c->alpha_z))
    return fail(EMAGPIE_E_ARG, "alpha_z must be finite and >= 0");
  if (c->update_probe != 0 && c->update_probe != 1) return fail(EMAGPIE_E_ARG, "update_probe must be 0 or 1");
  if (c->joint_step != 0 && c->joint_step != 1) return fail(EMAGPIE_E_ARG, "joint_step must be 0 or 1");
  if (c->path < EMAGPIE_PATH_PLAIN || c->path > EMAGPIE_PATH_CHAIN)
    return fail(EMAGPIE_E_ARG, "unknown path");
  if (c->path == EMAGPIE_PATH_CHAIN && c->minibatch != 1)
    return fail(EMAGPIE_E_ARG, "the chain path needs minibatch 1");
  if (c->zero_phase_memory != 0 && c->zero_phase_memory != 1)
    return fail(EMAGPIE_E_ARG, "zero_phase_memory must be 0 or 1");
  if (c->m == 256 && c->path != EMAGPIE_PATH_FUSED && c->path != EMAGPIE_PATH_GRAPH &&
      c->path != EMAGPIE_PATH_AUTO)
    return fail(EMAGPIE_E_UNSUPPORTED, "m = 256 runs the fused and graph paths only");
  if (c->fft_plan != EMAGPIE_TUNE && (c->fft_plan < 0 || c->fft_plan >= emg::fft_plan_count(c->m)))
    return fail(EMAGPIE_E_ARG, "fft_plan must be EMAGPIE_TUNE or in [0, " +
                                   std::to_string(emg::fft_plan_count(c->m)) + ") for this m");
  if (c->finalize_shape != EMAGPIE_TUNE && (c->finalize_shape < 0 || c->finalize_shape >= emg::kFinShapes))
    return fail(EMAGPIE_E_ARG, "finalize_shape must be EMAGPIE_TUNE or in [0, " +
                                   std::to_string(emg::kFinShapes) + ")");
  return EMAGPIE_OK;
}

}  // namespace

struct Many;  // members and group of a context made by emagpie_init_many

struct emagpie_ctx_s {
  emagpie_config cfg;  // path, fft_plan and finalize_shape hold the resolved choice
  Layout lay;
  int layout_plan = 0;  // FFT plan whose transform order dperm holds
  emagpie_plan plan{};
  uint8_t* ws;
  float* dperm;
  int2* pos;
  int4* slots;  // per slot of the current sweep / batch: (k, row, col, 0)
  int4* morder;  // every pattern, in the full misfit's launch order (m < 256)
  float2* tw32;
  double2* tw64;
  float2 *numer, *pnum, *stack;
  float *pden, *pden_slot, *zmax, *ubuf, *Dbuf;
  double *phi, *phi_all;
  double* scal_d;  // [0] dp sum, [1] scratch
  int* scal_i;     // [0] bad-data flag, [1] zero-probe flag
  float* qqmax;
  float2* phase = nullptr;  // zero-bin phase memory (N x m^2 unit phasors) or null
  std::vector<int32_t> pos_host;
  std::vector<int32_t> perm_host;
  double dp_avg = 0.0;
  int num_cus = 0;
  int num_xcc = 1;  // accelerator complex dies (each with its own L2)
  std::vector<int4> listing_tmp;
  int persist_grid = 0;
  unsigned* bar = nullptr;  // persistent-kernel barrier counter (grows monotonically)
  unsigned bar_base = 0;
  bool bar_ready = false;
  int4* perm_pinned[2] = {nullptr, nullptr};
  hipEvent_t perm_ev[2] = {nullptr, nullptr};
  int perm_slot = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  void* g_obj = nullptr;
  void* g_probe = nullptr;
  double* g_sampled = nullptr;
  // kernel timing (category 0 patch stage, 1 finalize, 2 persistent epoch)
  bool profile = false;
  std::vector<hipEvent_t> ev[3];
  size_t ev_used[3] = {0, 0, 0};
  // device-side error flag in host memory (fine-grained, mapped): a persistent
  // epoch's grid barrier that gave up waiting sets it; the next call reports it
  int* dev_err_host = nullptr;
  int* dev_err_dev = nullptr;
  unsigned spin_limit = kDefaultSpinLimit;
  unsigned bar_skew = 0;  // extra arrivals awaited (fault injection; 0 in normal use)
  std::string err;        // last failure of a call on this context
  // a context made by emagpie_init_many: its members and their group
  Many* many = nullptr;
};

namespace {

#define EMG_OK(expr)                      \
  do {                                    \
    emagpie_status st_ = (expr);          \
    if (st_ != EMAGPIE_OK) return st_;    \
  } while (0)

// Copies a failure raised during an entry point's call into its context (the
// message emagpie_last_error(ctx) returns).
struct CtxErrScope {
  emagpie_ctx c;
  uint64_t n0;
  explicit CtxErrScope(emagpie_ctx c_) : c(c_), n0(g_err_count) {}
  ~CtxErrScope() {
    if (c && g_err_count != n0) c->err = g_err;
  }
};

// Entry check of a call on a single-instance context: not null, not a
// many-context, and no device error pending from earlier work.  A pending error is
// returned (once) instead of doing the call; the persistent barrier counter is then
// re-zeroed before the next persistent epoch.
emagpie_status use_ctx(emagpie_ctx c) {
  if (!c) return fail(EMAGPIE_E_ARG, "null context");
  if (c->many)
    return fail(EMAGPIE_E_ARG, "a context made by emagpie_init_many takes emagpie_epoch_many; "
                               "use emagpie_many_member for per-instance calls");
  if (c->dev_err_host && __atomic_load_n(c->dev_err_host, __ATOMIC_ACQUIRE) != 0) {
    __atomic_store_n(c->dev_err_host, 0, __ATOMIC_RELEASE);
    c->bar_ready = false;
    return fail(EMAGPIE_E_HIP,
                "device error raised by earlier work on this context: a grid barrier of a persistent "
                "epoch gave up waiting for the other workgroups; the object and probe that epoch "
                "wrote are not valid");
  }
  return EMAGPIE_OK;
}

emg::StepArgs base_args(emagpie_ctx c, void* obj, void* probe) {
  emg::StepArgs a{};
  a.obj = static_cast<float2*>(obj);
  a.n = c->cfg.n_cols;
  a.nr = c->cfg.n_rows;
  a.probe = static_cast<float2*>(probe);
  a.dperm = c->dperm;
  a.pos = c->pos;
  a.alpha = c->cfg.alpha;
  a.alpha_z = c->cfg.alpha_z;
  a.update_probe = c->cfg.update_probe;
  a.joint = c->cfg.joint_step;
  a.pgroups = emg::probe_groups(c->cfg.minibatch);
  a.phase = c->phase;
  a.phase_write = 1;
  if (c->cfg.m == 256) {
    uint8_t* p = c->ws + c->lay.part.off;
    const size_t B = (size_t)c->cfg.minibatch;
    a.part_q = reinterpret_cast<float*>(p);
    a.part_z = reinterpret_cast<float*>(p + B * 16 * 4);
    a.part_phi = reinterpret_cast<double*>(p + B * 16 * 8);
  }
  a.tw = c->tw32;
  a.numer = c->numer;
  a.pnum = c->pnum;
  a.pden = c->pden;
  // alpha_z = 1 (the ePIE probe step): |z_k|^2 + u_z = max |z_k|^2, one value per patch
  a.pden_slot = c->cfg.alpha_z == 1.0f ? c->pden_slot : nullptr;
  a.phi = c->phi;
  a.Dbuf = c->Dbuf;
  a.stack = c->stack;
  a.zmax = c->zmax;
  a.ubuf = c->ubuf;
  a.qqmax = c->qqmax;
  return a;
}

// a (start, stop) event pair for timing category `cat`, or nulls when not timing
emagpie_status take_pair(emagpie_ctx c, int cat, bool instrument, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!c->profile || !instrument) return EMAGPIE_OK;
  while (c->ev[cat].size() < c->ev_used[cat] + 2) {
    hipEvent_t e;
    EMG_HIP(hipEventCreate(&e));
    c->ev[cat].push_back(e);
  }
  *e0 = c->ev[cat][c->ev_used[cat]++];
  *e1 = c->ev[cat][c->ev_used[cat]++];
  return EMAGPIE_OK;
}

// enqueue one minibatch with the configured (non-graph) strategy
emagpie_status enqueue_minibatch(emagpie_ctx c, const emg::StepArgs& a, bool plain, hipStream_t s,
                                 bool instrument = true) {
  const int m = c->cfg.m, L = c->cfg.levels;
  hipEvent_t e0, e1;
  EMG_OK(take_pair(c, 0, instrument, &e0, &e1));
  if (plain) {
    // six kernels: the pair brackets the group on the stream
    if (e0) EMG_HIP(hipEventRecord(e0, s));
    EMG_HIP(emg::launch_plain_step(m, c->cfg.fft_plan, L, a, s));
    if (e1) EMG_HIP(hipEventRecord(e1, s));
  } else {
    EMG_HIP(emg::launch_patch_step(m, c->cfg.fft_plan, L, a, s, e0, e1));
  }
  EMG_OK(take_pair(c, 1, instrument, &e0, &e1));
  EMG_HIP(emg::launch_finalize(m, c->cfg.finalize_shape, a, s, e0, e1));
  return EMAGPIE_OK;
}

emagpie_status enqueue_sweep(emagpie_ctx c, void* obj, void* probe, double* sampled, bool plain,
                             hipStream_t s, bool instrument = true) {
  if (sampled) EMG_HIP(emg::launch_zero_doubles(sampled, 1, s));
  const int N = c->cfg.n_pos, B = c->cfg.minibatch;
  for (int start = 0; start < N; start += B) {
    emg::StepArgs a = base_args(c, obj, probe);
    a.slot = c->slots + start;
    a.b = std::min(B, N - start);
    a.sampled = sampled;
    emagpie_status st = enqueue_minibatch(c, a, plain, s, instrument);
    if (st != EMAGPIE_OK) return st;
  }
  return EMAGPIE_OK;
}

void drop_graph(emagpie_ctx c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}


// ---------------------------------------------------------------------------
// autotuning at init
// ---------------------------------------------------------------------------
void fill_plan_info(emagpie_ctx c, int tuned) {
  emagpie_plan& p = c->plan;
  p.fft_plan = c->cfg.fft_plan;
  emg::fft_plan_desc(c->cfg.m, p.fft_plan, &p.r1, &p.r2, &p.threads);
  p.finalize_shape = c->cfg.finalize_shape;
  emg::fin_shape_desc(p.finalize_shape, &p.fin_threads, &p.fin_tile, &p.fin_order);
  p.path = c->cfg.path;
  p.tuned = tuned;
  if (tuned == 0) {
    p.n_fft_plans = p.n_fin_shapes = 0;
    for (float& x : p.fft_us) x = -1.f;
    for (float& x : p.fin_us) x = -1.f;
    for (float& x : p.path_ms) x = -1.f;
  }
}

std::string tune_key(emagpie_ctx c, const emagpie_config& req) {
  hipDeviceProp_t prop{};
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  const emagpie_config& k = c->cfg;
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "%s cus=%d m=%d n=%dx%d N=%d B=%d L=%d blind=%d joint=%d az1=%d mem=%d plan=%d "
                "shape=%d path=%d",
                arch.c_str(), c->num_cus, k.m, k.n_rows, k.n_cols, k.n_pos, k.minibatch, k.levels, k.update_probe,
                k.joint_step, k.alpha_z == 1.0f ? 1 : 0, k.zero_phase_memory, req.fft_plan,
                req.finalize_shape, req.path);
  return buf;
}

bool json_int(const std::string& line, const char* name, int* out) {
  const std::string pat = std::string("\"") + name + "\": ";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return false;
  char* end = nullptr;
  const long v = std::strtol(line.c_str() + at + pat.size(), &end, 10);
  if (end == line.c_str() + at + pat.size()) return false;
  *out = (int)v;
  return true;
}

// last line of the cache whose key matches; false if none (or unreadable)
bool cache_lookup(const char* path, const std::string& key, int* v, int* f, int* p) {
  if (!path) return false;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  bool found = false;
  const std::string kpat = "\"key\": \"" + key + "\"";
  char buf[4096];
  while (std::fgets(buf, sizeof buf, fp)) {
    const std::string line(buf);
    if (line.find(kpat) == std::string::npos) continue;
    int a, b, q;
    if (json_int(line, "fft_plan", &a) && json_int(line, "finalize_shape", &b) &&
        json_int(line, "path", &q)) {
      *v = a;
      *f = b;
      *p = q;
      found = true;
    }
  }
  std::fclose(fp);
  return found;
}

void cache_append(const char* path, const std::string& key, const emagpie_plan& p) {
  if (!path) return;
  FILE* fp = std::fopen(path, "a");
  if (!fp) return;
  auto arr = [](const float* x, int n) {
    std::string r = "[";
    for (int i = 0; i < n; ++i) {
      char b[32];
      std::snprintf(b, sizeof b, "%s%.4g", i ? ", " : "", x[i]);
      r += b;
    }
    return r + "]";
  };
  std::fprintf(fp,
               "{\"key\": \"%s\", \"fft_plan\": %d, \"finalize_shape\": %d, \"path\": %d, "
               "\"fft_us\": %s, \"fin_us\": %s, \"path_ms\": %s}\n",
               key.c_str(), p.fft_plan, p.finalize_shape, p.path, arr(p.fft_us, 4).c_str(),
               arr(p.fin_us, emg::kFinShapes).c_str(), arr(p.path_ms, 6).c_str());
  std::fclose(fp);
}

// Lay the intensities out in the transform order of FFT plan v (if the
// current layout's radix split differs).
emagpie_status relayout(emagpie_ctx c, int v, const float* intensities_dev, hipStream_t s) {
  int r1a, r2a, nta, r1b, r2b, ntb;
  emg::fft_plan_desc(c->cfg.m, c->layout_plan, &r1a, &r2a, &nta);
  emg::fft_plan_desc(c->cfg.m, v, &r1b, &r2b, &ntb);
  if (r1a != r1b || r2a != r2b) {
    EMG_HIP(emg::launch_layout_intensities(c->cfg.m, v, intensities_dev, c->dperm, c->cfg.n_pos,
                                           c->phi_all, c->scal_i + 3, s));
  }
  c->layout_plan = v;
  return EMAGPIE_OK;
}

float median(std::vector<float> x) {
  std::sort(x.begin(), x.end());
  return x.empty() ? -1.f : x[x.size() / 2];
}

// Time `reps` launches made by enq(rep, e0, e1) (each brackets its timed kernel
// with the events) after `warm` untimed ones; median milliseconds.
template <class Enq>
emagpie_status time_kernel(hipStream_t s, int warm, int reps, Enq enq, float* ms_out) {
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  emagpie_status st = EMAGPIE_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) st = fail(EMAGPIE_E_HIP, "tuner event");
  for (int i = 0; st == EMAGPIE_OK && i < warm; ++i) st = enq(i, nullptr, nullptr);
  for (int i = 0; st == EMAGPIE_OK && i < reps; ++i) st = enq(warm + i, ev[2 * i], ev[2 * i + 1]);
  if (st == EMAGPIE_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(EMAGPIE_E_HIP, "tuner sync");
  std::vector<float> ms;
  for (int i = 0; st == EMAGPIE_OK && i < reps; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) != hipSuccess)
      st = fail(EMAGPIE_E_HIP, "tuner timing");
    ms.push_back(t);
  }
  (void)hipStreamSynchronize(s);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  *ms_out = median(ms);
  return st;
}

emagpie_status autotune(emagpie_ctx c, const emagpie_config& req, const float* intensities_dev,
                        hipStream_t s) {
  const int m = c->cfg.m, N = c->cfg.n_pos, B = c->cfg.minibatch, L = c->cfg.levels;
  const std::string key = tune_key(c, req);
  int cv, cf, cp;
  if (cache_lookup(req.tune_cache, key, &cv, &cf, &cp) && cv >= 0 && cv < emg::fft_plan_count(m) &&
      cf >= 0 && cf < emg::kFinShapes && cp >= EMAGPIE_PATH_PLAIN && cp <= EMAGPIE_PATH_CHAIN &&
      cp != EMAGPIE_PATH_AUTO && (cp != EMAGPIE_PATH_CHAIN || B == 1)) {
    EMG_OK(relayout(c, cv, intensities_dev, s));
    c->cfg.fft_plan = cv;
    c->cfg.finalize_shape = cf;
    c->cfg.path = cp;
    EMG_HIP(emg::persistent_grid_size(m, cv, L, c->num_cus, &c->persist_grid));
    EMG_HIP(hipStreamSynchronize(s));
    fill_plan_info(c, 2);
    return EMAGPIE_OK;
  }
  emagpie_plan& P = c->plan;
  // scratch state (unit object, unit probe) and the epoch-0 scan order
  float2* tobj = reinterpret_cast<float2*>(c->ws + c->lay.tune_obj.off);
  float2* tprobe = reinterpret_cast<float2*>(c->ws + c->lay.tune_probe.off);
  EMG_HIP(emg::launch_fill_c64(tobj, (size_t)c->cfg.n_rows * c->cfg.n_cols, make_float2(1.f, 0.f), s));
  EMG_HIP(emg::launch_fill_c64(tprobe, (size_t)m * m, make_float2(1.f, 0.f), s));
  std::vector<int32_t> perm(N);
  fisher_yates(c->cfg.seed, 0, N, perm.data());
  int4* pin = c->perm_pinned[0];
  for (int j = 0; j < N; ++j) {
    const int k = perm[j];
    pin[j] = make_int4(k, c->pos_host[2 * k], c->pos_host[2 * k + 1], 0);
  }
  xcd_listing_sweep(pin, N, std::min(B, N), c->num_xcc, c->listing_tmp);
  EMG_HIP(hipMemcpyAsync(c->slots, pin, sizeof(int4) * N, hipMemcpyHostToDevice, s));
  EMG_HIP(hipStreamSynchronize(s));
  const int b = std::min(B, N), nb = std::max(1, N / b);
  auto batch_args = [&](int rep) {
    emg::StepArgs a = base_args(c, tobj, tprobe);
    a.slot = c->slots + (size_t)(rep % nb) * b;
    a.b = b;
    return a;
  };
  constexpr int kWarm = 2, kReps = 11;

  // 1. FFT plan: time the patch-stage kernel of every candidate
  if (req.fft_plan == EMAGPIE_TUNE) {
    const int nv = emg::fft_plan_count(m);
    P.n_fft_plans = nv;
    int best = 0;
    for (int v = 0; v < nv; ++v) {
      EMG_OK(relayout(c, v, intensities_dev, s));
      float ms = -1.f;
      EMG_OK(time_kernel(s, kWarm, kReps, [&](int rep, hipEvent_t e0, hipEvent_t e1) -> emagpie_status {
        EMG_HIP(emg::launch_patch_step(m, v, L, batch_args(rep), s, e0, e1));
        return EMAGPIE_OK;
      }, &ms));
      P.fft_us[v] = 1000.f * ms;
      if (P.fft_us[v] < P.fft_us[best]) best = v;
    }
    EMG_OK(relayout(c, best, intensities_dev, s));
    c->cfg.fft_plan = best;
    EMG_HIP(emg::persistent_grid_size(m, best, L, c->num_cus, &c->persist_grid));
  }
  // 2. finalize shape: time the finalize after an untimed patch stage
  if (req.finalize_shape == EMAGPIE_TUNE) {
    P.n_fin_shapes = emg::kFinShapes;
    int best = 0;
    for (int f = 0; f < emg::kFinShapes; ++f) {
      float ms = -1.f;
      EMG_OK(time_kernel(s, kWarm, kReps, [&](int rep, hipEvent_t e0, hipEvent_t e1) -> emagpie_status {
        const emg::StepArgs a = batch_args(rep);
        EMG_HIP(emg::launch_patch_step(m, c->cfg.fft_plan, L, a, s));
        EMG_HIP(emg::launch_finalize(m, f, a, s, e0, e1));
        return EMAGPIE_OK;
      }, &ms));
      P.fin_us[f] = 1000.f * ms;
      if (P.fin_us[f] < P.fin_us[best]) best = f;
    }
    // The two fastest shapes alone can rank the other way inside an epoch (the
    // finalize leaves the caches to the next patch stage): the fused epoch decides.
    static_assert(emg::kFinShapes >= 2, "two finalize shapes to compare");
    static_assert(sizeof(P.fin_us) / sizeof(P.fin_us[0]) >= emg::kFinShapes, "room for every shape");
    int second = best == 0 ? 1 : 0;
    for (int f = 0; f < emg::kFinShapes; ++f)
      if (f != best && P.fin_us[f] < P.fin_us[second]) second = f;
    const int saved_path = c->cfg.path;
    c->cfg.path = EMAGPIE_PATH_FUSED;
    float ep[2] = {0.f, 0.f};
    const int pair[2] = {best, second};
    int64_t epoch = 0;
    for (int i = 0; i < 2; ++i) {
      c->cfg.finalize_shape = pair[i];
      EMG_OK(time_kernel(s, 1, 3, [&](int, hipEvent_t e0, hipEvent_t e1) -> emagpie_status {
        if (e0) EMG_HIP(hipEventRecord(e0, s));
        EMG_OK(emagpie_epoch(c, tobj, tprobe, epoch++, nullptr, nullptr, s));
        if (e1) EMG_HIP(hipEventRecord(e1, s));
        return EMAGPIE_OK;
      }, &ep[i]));
    }
    c->cfg.path = saved_path;
    c->cfg.finalize_shape = ep[1] < ep[0] ? second : best;
  }
  // 3. path: whole epochs on the scratch state.  The persistent path is not a
  // candidate: it was slower on every workload measured, and its cooperative launch
  // leaves the process's later launches slower (most of all concurrent graph branches,
  // as in a group sweep), so timing it here would cost the path that wins.
  if (req.path == EMAGPIE_PATH_AUTO) {
    const int cand[3] = {EMAGPIE_PATH_FUSED, EMAGPIE_PATH_GRAPH, EMAGPIE_PATH_CHAIN};
    int best = EMAGPIE_PATH_FUSED;
    for (int p : cand) {
      if (p == EMAGPIE_PATH_CHAIN && B != 1) continue;
      if (m == 256 && p != EMAGPIE_PATH_FUSED && p != EMAGPIE_PATH_GRAPH) continue;
      c->cfg.path = p;
      float ms = -1.f;
      int64_t epoch = 0;
      EMG_OK(time_kernel(s, 1, 3, [&](int, hipEvent_t e0, hipEvent_t e1) -> emagpie_status {
        if (e0) EMG_HIP(hipEventRecord(e0, s));
        EMG_OK(emagpie_epoch(c, tobj, tprobe, epoch++, nullptr, nullptr, s));
        if (e1) EMG_HIP(hipEventRecord(e1, s));
        return EMAGPIE_OK;
      }, &ms));
      P.path_ms[p] = ms;
      if (P.path_ms[p] < P.path_ms[best]) best = p;
    }
    c->cfg.path = best;
    drop_graph(c);
  }
  // the timed runs wrote phasors of the scratch state: back to the first-sweep state
  if (c->phase)
    EMG_HIP(emg::launch_fill_c64(c->phase, (size_t)N * m * m, make_float2(1.f, 0.f), s));
  EMG_HIP(hipStreamSynchronize(s));
  fill_plan_info(c, 1);
  cache_append(req.tune_cache, key, P);
  return EMAGPIE_OK;
}

}  // namespace

extern "C" {

const char* emagpie_version(void) { return "libemagpie 0.1 (gfx950)"; }

const char* emagpie_last_error(emagpie_ctx ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

emagpie_status emagpie_workspace_size(const emagpie_config* cfg, size_t* bytes) {
  emagpie_status st = check_config(cfg);
  if (st != EMAGPIE_OK) return st;
  if (!bytes) return fail(EMAGPIE_E_ARG, "null output");
  *bytes = make_layout(*cfg).total;
  return EMAGPIE_OK;
}

emagpie_status emagpie_permutation(uint64_t seed, int64_t epoch, int32_t n, int32_t* out_host) {
  if (n < 0 || (n > 0 && !out_host)) return fail(EMAGPIE_E_ARG, "bad permutation arguments");
  fisher_yates(seed, epoch, n, out_host);
  return EMAGPIE_OK;
}

emagpie_status emagpie_init(emagpie_ctx* out, const emagpie_config* cfg,
                            const int32_t* positions_host, const float* intensities_dev,
                            void* workspace_dev, size_t workspace_bytes, void* stream) {
  if (!out) return fail(EMAGPIE_E_ARG, "null context output");
  *out = nullptr;
  emagpie_status st = check_config(cfg);
  if (st != EMAGPIE_OK) return st;
  if (!positions_host || !intensities_dev) return fail(EMAGPIE_E_ARG, "null positions or intensities");
  const emagpie_config c = *cfg;
  for (int k = 0; k < c.n_pos; ++k) {
    const int32_t r = positions_host[2 * k], q = positions_host[2 * k + 1];
    if (r < 0 || q < 0 || r > c.n_rows - c.m || q > c.n_cols - c.m)
      return fail(EMAGPIE_E_POSITION, "scan position " + std::to_string(k) + " = (" +
                                          std::to_string(r) + ", " + std::to_string(q) +
                                          ") leaves the object");
  }
  const Layout lay = make_layout(c);
  if (!workspace_dev || (reinterpret_cast<uintptr_t>(workspace_dev) & 255))
    return fail(EMAGPIE_E_WORKSPACE, "workspace missing or not 256-byte aligned");
  if (workspace_bytes < lay.total)
    return fail(EMAGPIE_E_WORKSPACE, "workspace too small: need " + std::to_string(lay.total) +
                                         " bytes, got " + std::to_string(workspace_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);

  auto* ctx = new emagpie_ctx_s();
  ctx->cfg = c;
  ctx->lay = lay;
  uint8_t* w = static_cast<uint8_t*>(workspace_dev);
  ctx->ws = w;
  ctx->dperm = reinterpret_cast<float*>(w + lay.dperm.off);
  ctx->pos = reinterpret_cast<int2*>(w + lay.pos.off);
  ctx->slots = reinterpret_cast<int4*>(w + lay.slots.off);
  ctx->morder = reinterpret_cast<int4*>(w + lay.morder.off);
  ctx->tw32 = reinterpret_cast<float2*>(w + lay.tw32.off);
  ctx->tw64 = reinterpret_cast<double2*>(w + lay.tw64.off);
  ctx->numer = reinterpret_cast<float2*>(w + lay.numer.off);
  ctx->pnum = reinterpret_cast<float2*>(w + lay.pnum.off);
  ctx->pden = reinterpret_cast<float*>(w + lay.pden.off);
  ctx->pden_slot = reinterpret_cast<float*>(w + lay.pden_slot.off);
  ctx->phi = reinterpret_cast<double*>(w + lay.phi.off);
  ctx->stack = reinterpret_cast<float2*>(w + lay.stack.off);
  ctx->zmax = reinterpret_cast<float*>(w + lay.zmax.off);
  ctx->ubuf = reinterpret_cast<float*>(w + lay.ubuf.off);
  ctx->Dbuf = reinterpret_cast<float*>(w + lay.Dbuf.off);
  ctx->scal_d = reinterpret_cast<double*>(w + lay.scal.off);
  ctx->scal_i = reinterpret_cast<int*>(w + lay.scal.off + 64);
  ctx->qqmax = reinterpret_cast<float*>(w + lay.scal.off + 128);
  ctx->phi_all = reinterpret_cast<double*>(w + lay.phi_all.off);
  ctx->bar = reinterpret_cast<unsigned*>(w + lay.bar.off);
  if (c.zero_phase_memory) ctx->phase = reinterpret_cast<float2*>(w + lay.phase.off);
  ctx->pos_host.assign(positions_host, positions_host + 2 * (size_t)c.n_pos);

  auto bail = [&](emagpie_status e) {
    emagpie_destroy(ctx);
    return e;
  };
  auto hipfail = [&](hipError_t e, const char* what) {
    fail(EMAGPIE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return bail(EMAGPIE_E_HIP);
  };
  hipError_t e;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hipfail(e, "hipGetDevice");
  if ((e = hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hipfail(e, "hipDeviceGetAttribute");
  if (hipDeviceGetAttribute(&ctx->num_xcc, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess ||
      ctx->num_xcc < 1)
    ctx->num_xcc = 1;
  // the plan the context starts with: the configured one, or the defaults
  // until the autotuner below has chosen
  if (ctx->cfg.fft_plan == EMAGPIE_TUNE) ctx->cfg.fft_plan = 0;
  if (ctx->cfg.finalize_shape == EMAGPIE_TUNE) ctx->cfg.finalize_shape = 0;
  if (ctx->cfg.path == EMAGPIE_PATH_AUTO) ctx->cfg.path = EMAGPIE_PATH_FUSED;
  ctx->layout_plan = ctx->cfg.fft_plan;
  if ((e = emg::persistent_grid_size(c.m, ctx->cfg.fft_plan, c.levels, ctx->num_cus,
                                     &ctx->persist_grid)) != hipSuccess)
    return hipfail(e, "occupancy query");

  // twiddles exp(-2 pi i j / m), evaluated in double on the host
  std::vector<float2> t32(c.m);
  std::vector<double2> t64(c.m);
  for (int j = 0; j < c.m; ++j) {
    const double ang = -2.0 * M_PI * (double)j / (double)c.m;
    const double cr = std::cos(ang), ci = std::sin(ang);
    t32[j] = make_float2((float)cr, (float)ci);
    t64[j] = make_double2(cr, ci);
  }
  std::vector<int2> p2(c.n_pos);
  for (int k = 0; k < c.n_pos; ++k) p2[k] = make_int2(positions_host[2 * k], positions_host[2 * k + 1]);
  if ((e = hipMemcpyAsync(ctx->tw32, t32.data(), c.m * sizeof(float2), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hipfail(e, "upload twiddles");
  if ((e = hipMemcpyAsync(ctx->tw64, t64.data(), c.m * sizeof(double2), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hipfail(e, "upload twiddles");
  if ((e = hipMemcpyAsync(ctx->pos, p2.data(), c.n_pos * sizeof(int2), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hipfail(e, "upload positions");
  std::vector<int4> order;
  if (c.m != 256) {
    misfit_order(positions_host, c.n_pos, ctx->num_xcc, order);
    if ((e = hipMemcpyAsync(ctx->morder, order.data(), c.n_pos * sizeof(int4), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
      return hipfail(e, "upload misfit order");
  }
  if ((e = hipMemsetAsync(ctx->scal_i, 0, 64, s)) != hipSuccess) return hipfail(e, "clear flags");
  if (ctx->phase &&
      (e = emg::launch_fill_c64(ctx->phase, (size_t)c.n_pos * c.m * c.m, make_float2(1.f, 0.f), s)) !=
          hipSuccess)
    return hipfail(e, "clear phase memory");
  if ((e = emg::launch_layout_intensities(c.m, ctx->layout_plan, intensities_dev, ctx->dperm, c.n_pos,
                                           ctx->phi_all,
                                           ctx->scal_i, s)) != hipSuccess)
    return hipfail(e, "layout intensities");
  if ((e = emg::launch_sum_doubles(ctx->phi_all, c.n_pos, ctx->scal_d, s)) != hipSuccess)
    return hipfail(e, "sum intensities");
  double total = 0.0;
  int bad = 0;
  if ((e = hipMemcpyAsync(&total, ctx->scal_d, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hipfail(e, "read sum");
  if ((e = hipMemcpyAsync(&bad, ctx->scal_i, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hipfail(e, "read flag");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hipfail(e, "synchronise init");
  if (bad) {
    fail(EMAGPIE_E_DATA, "intensities contain NaN or Inf");
    return bail(EMAGPIE_E_DATA);
  }
  ctx->dp_avg = std::sqrt(total / (double)c.n_pos) / (double)c.m;

  for (int i = 0; i < 2; ++i) {
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&ctx->perm_pinned[i]), sizeof(int4) * c.n_pos,
                           hipHostMallocDefault)) != hipSuccess)
      return hipfail(e, "pinned permutation buffer");
    if ((e = hipEventCreateWithFlags(&ctx->perm_ev[i], hipEventDisableTiming)) != hipSuccess)
      return hipfail(e, "event");
  }
  // the device-side error flag: fine-grained host memory the kernels can write and
  // the host can read at its next call without synchronising
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&ctx->dev_err_host), 64,
                         hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
    return hipfail(e, "device error flag");
  __atomic_store_n(ctx->dev_err_host, 0, __ATOMIC_RELEASE);
  if ((e = hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->dev_err_dev), ctx->dev_err_host, 0)) !=
      hipSuccess)
    return hipfail(e, "device error flag mapping");
  fill_plan_info(ctx, 0);
  if (wants_tuning(c)) {
    emagpie_status ts = autotune(ctx, c, intensities_dev, s);
    if (ts != EMAGPIE_OK) return bail(ts);
  }
  ctx->cfg.tune_cache = nullptr;  // the caller's string is only read during init
  *out = ctx;
  g_err.clear();
  return EMAGPIE_OK;
}

emagpie_status emagpie_phase_memory_reset(emagpie_ctx ctx, void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!ctx->phase) return fail(EMAGPIE_E_ARG, "the context has no phase memory");
  EMG_HIP(emg::launch_fill_c64(ctx->phase, (size_t)ctx->cfg.n_pos * ctx->cfg.m * ctx->cfg.m,
                               make_float2(1.f, 0.f), static_cast<hipStream_t>(stream)));
  return EMAGPIE_OK;
}

emagpie_status emagpie_plan_get(emagpie_ctx ctx, emagpie_plan* out_host) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!out_host) return fail(EMAGPIE_E_ARG, "null argument");
  *out_host = ctx->plan;
  return EMAGPIE_OK;
}

emagpie_status emagpie_plan_describe(int32_t m, int32_t fft_plan, int32_t finalize_shape,
                                     emagpie_plan* out_host, int32_t* count_host) {
  if (count_host) *count_host = emg::fft_plan_count(m);
  if (!out_host) return fail(EMAGPIE_E_ARG, "null output");
  emagpie_plan p{};
  if (!emg::fft_plan_desc(m, fft_plan, &p.r1, &p.r2, &p.threads))
    return fail(EMAGPIE_E_ARG, "no such FFT plan for this m");
  if (!emg::fin_shape_desc(finalize_shape, &p.fin_threads, &p.fin_tile, &p.fin_order))
    return fail(EMAGPIE_E_ARG, "no such finalize shape");
  p.fft_plan = fft_plan;
  p.finalize_shape = finalize_shape;
  p.path = -1;
  for (float& x : p.path_ms) x = -1.f;
  *out_host = p;
  return EMAGPIE_OK;
}

emagpie_status emagpie_profile_enable(emagpie_ctx ctx, int32_t enable) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  ctx->profile = enable != 0;
  return EMAGPIE_OK;
}

emagpie_status emagpie_profile_read(emagpie_ctx ctx, double* ms3_host, int64_t* count3_host) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!ms3_host || !count3_host) return fail(EMAGPIE_E_ARG, "null argument");
  for (int cat = 0; cat < 3; ++cat) {
    double tot = 0.0;
    const size_t used = ctx->ev_used[cat];
    for (size_t i = 0; i + 1 < used; i += 2) {
      EMG_HIP(hipEventSynchronize(ctx->ev[cat][i + 1]));
      float ms = 0.f;
      EMG_HIP(hipEventElapsedTime(&ms, ctx->ev[cat][i], ctx->ev[cat][i + 1]));
      tot += ms;
    }
    ms3_host[cat] = tot;
    count3_host[cat] = (int64_t)(used / 2);
    ctx->ev_used[cat] = 0;
  }
  return EMAGPIE_OK;
}

void destroy_many(emagpie_ctx ctx);

emagpie_status emagpie_destroy(emagpie_ctx ctx) {
  if (!ctx) return EMAGPIE_OK;
  if (ctx->many) {
    destroy_many(ctx);
    return EMAGPIE_OK;
  }
  drop_graph(ctx);
  for (int cat = 0; cat < 3; ++cat) {
    for (hipEvent_t e : ctx->ev[cat]) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (int i = 0; i < 2; ++i) {
    if (ctx->perm_ev[i]) {
      (void)hipEventSynchronize(ctx->perm_ev[i]);
      (void)hipEventDestroy(ctx->perm_ev[i]);
    }
    if (ctx->perm_pinned[i]) (void)hipHostFree(ctx->perm_pinned[i]);
  }
  if (ctx->dev_err_host) (void)hipHostFree(ctx->dev_err_host);
  delete ctx;
  return EMAGPIE_OK;
}

emagpie_status emagpie_dp_avg(emagpie_ctx ctx, double* dp_avg_host) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!dp_avg_host) return fail(EMAGPIE_E_ARG, "null argument");
  *dp_avg_host = ctx->dp_avg;
  return EMAGPIE_OK;
}

emagpie_status emagpie_normalize_probe(emagpie_ctx ctx, void* probe_dev, void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!probe_dev) return fail(EMAGPIE_E_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int flag = 0;
  EMG_HIP(hipMemsetAsync(ctx->scal_i + 1, 0, sizeof(int), s));
  EMG_HIP(emg::launch_normalize_probe(ctx->cfg.m, static_cast<float2*>(probe_dev), ctx->dp_avg,
                                      ctx->scal_i + 1, s));
  EMG_HIP(hipMemcpyAsync(&flag, ctx->scal_i + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  EMG_HIP(hipStreamSynchronize(s));
  if (flag) return fail(EMAGPIE_E_DEGENERATE, "probe is zero; cannot normalise");
  return EMAGPIE_OK;
}

emagpie_status emagpie_step_minibatch(emagpie_ctx ctx, void* obj_dev, void* probe_dev,
                                      const int32_t* batch_idx_dev, int32_t b,
                                      double* sampled_misfit_dev, void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!obj_dev || !probe_dev || !batch_idx_dev) return fail(EMAGPIE_E_ARG, "null argument");
  if (b < 1 || b > ctx->cfg.minibatch) return fail(EMAGPIE_E_ARG, "b must be in [1, minibatch]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  EMG_HIP(emg::launch_slot_info(batch_idx_dev, ctx->pos, ctx->cfg.n_pos, ctx->slots, b, s));
  emg::StepArgs a = base_args(ctx, obj_dev, probe_dev);
  a.slot = ctx->slots;
  a.b = b;
  a.sampled = sampled_misfit_dev;
  if (ctx->cfg.path == EMAGPIE_PATH_CHAIN) {
    if (sampled_misfit_dev) EMG_HIP(emg::launch_zero_doubles(sampled_misfit_dev, 1, s));
    EMG_HIP(emg::launch_chain_sweep(ctx->cfg.m, ctx->cfg.fft_plan, ctx->cfg.levels, a, b, s));
    return EMAGPIE_OK;
  }
  return enqueue_minibatch(ctx, a, ctx->cfg.path == EMAGPIE_PATH_PLAIN, s);
}

emagpie_status emagpie_epoch(emagpie_ctx ctx, void* obj_dev, void* probe_dev, int64_t epoch,
                             const int32_t* perm_dev, double* sampled_misfit_dev, void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!obj_dev || !probe_dev) return fail(EMAGPIE_E_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int N = ctx->cfg.n_pos;
  if (perm_dev) {
    EMG_HIP(emg::launch_slot_info(perm_dev, ctx->pos, N, ctx->slots, N, s));
  } else {
    // scan order and window corners gathered on the host, one upload per sweep
    const int slot = ctx->perm_slot;
    ctx->perm_slot ^= 1;
    EMG_HIP(hipEventSynchronize(ctx->perm_ev[slot]));  // the copy that last read this buffer
    ctx->perm_host.resize(N);
    fisher_yates(ctx->cfg.seed, epoch, N, ctx->perm_host.data());
    int4* dst = ctx->perm_pinned[slot];
    for (int j = 0; j < N; ++j) {
      const int k = ctx->perm_host[j];
      dst[j] = make_int4(k, ctx->pos_host[2 * k], ctx->pos_host[2 * k + 1], 0);
    }
    xcd_listing_sweep(dst, N, std::min(ctx->cfg.minibatch, N), ctx->num_xcc, ctx->listing_tmp);
    EMG_HIP(hipMemcpyAsync(ctx->slots, dst, sizeof(int4) * N, hipMemcpyHostToDevice, s));
    EMG_HIP(hipEventRecord(ctx->perm_ev[slot], s));
  }
  switch (ctx->cfg.path) {
    case EMAGPIE_PATH_PLAIN:
      return enqueue_sweep(ctx, obj_dev, probe_dev, sampled_misfit_dev, true, s);
    case EMAGPIE_PATH_FUSED:
      return enqueue_sweep(ctx, obj_dev, probe_dev, sampled_misfit_dev, false, s);
    case EMAGPIE_PATH_GRAPH: {
      if (!ctx->gexec || ctx->g_obj != obj_dev || ctx->g_probe != probe_dev ||
          ctx->g_sampled != sampled_misfit_dev) {
        drop_graph(ctx);
        if (!ctx->cap_stream) EMG_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        EMG_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        emagpie_status st =
            enqueue_sweep(ctx, obj_dev, probe_dev, sampled_misfit_dev, false, ctx->cap_stream, false);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &g);
        if (st != EMAGPIE_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (ec != hipSuccess) return fail(EMAGPIE_E_HIP, std::string("capture: ") + hipGetErrorString(ec));
        ctx->graph = g;
        EMG_HIP(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
        ctx->g_obj = obj_dev;
        ctx->g_probe = probe_dev;
        ctx->g_sampled = sampled_misfit_dev;
      }
      EMG_HIP(hipGraphLaunch(ctx->gexec, s));
      return EMAGPIE_OK;
    }
    case EMAGPIE_PATH_CHAIN: {
      if (sampled_misfit_dev) EMG_HIP(emg::launch_zero_doubles(sampled_misfit_dev, 1, s));
      emg::StepArgs a = base_args(ctx, obj_dev, probe_dev);
      a.slot = ctx->slots;
      a.b = 1;
      a.sampled = sampled_misfit_dev;
      hipEvent_t e0, e1;
      EMG_OK(take_pair(ctx, 2, true, &e0, &e1));
      if (e0) EMG_HIP(hipEventRecord(e0, s));
      EMG_HIP(emg::launch_chain_sweep(ctx->cfg.m, ctx->cfg.fft_plan, ctx->cfg.levels, a, N, s));
      if (e1) EMG_HIP(hipEventRecord(e1, s));
      return EMAGPIE_OK;
    }
    case EMAGPIE_PATH_PERSISTENT: {
      if (sampled_misfit_dev) EMG_HIP(emg::launch_zero_doubles(sampled_misfit_dev, 1, s));
      emg::StepArgs a = base_args(ctx, obj_dev, probe_dev);
      a.slot = ctx->slots;
      a.b = std::min(ctx->cfg.minibatch, N);
      a.sampled = sampled_misfit_dev;
      if (!ctx->bar_ready || ctx->bar_base > (1u << 30)) {
        EMG_HIP(emg::launch_zero_u32(ctx->bar, s));
        ctx->bar_base = 0;
        ctx->bar_ready = true;
      }
      int used = 0;
      hipEvent_t e0, e1;
      EMG_OK(take_pair(ctx, 2, true, &e0, &e1));
      if (e0) EMG_HIP(hipEventRecord(e0, s));
      EMG_HIP(emg::launch_persistent_epoch(ctx->cfg.m, ctx->cfg.fft_plan, ctx->cfg.levels, a, N,
                                           ctx->cfg.minibatch,
                                           ctx->persist_grid, ctx->bar, ctx->bar_base + ctx->bar_skew,
                                           ctx->dev_err_dev, ctx->spin_limit, &used, s));
      if (e1) EMG_HIP(hipEventRecord(e1, s));
      // every workgroup arrives once at each of the 2 barriers of each minibatch, also
      // when a wait gives up (the device error then re-zeroes the counter first)
      const unsigned nbatch = (unsigned)((N + ctx->cfg.minibatch - 1) / ctx->cfg.minibatch);
      ctx->bar_base += 2u * nbatch * (unsigned)used;
      return EMAGPIE_OK;
    }
    default:
      return fail(EMAGPIE_E_ARG, "unknown path");
  }
}

emagpie_status emagpie_mg_cycle(emagpie_ctx ctx, const void* obj_dev, const void* probe_dev,
                                const int32_t* batch_idx_dev, int32_t b, void* zplus_dev,
                                void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!obj_dev || !probe_dev || !batch_idx_dev || !zplus_dev)
    return fail(EMAGPIE_E_ARG, "null argument");
  if (b < 1 || b > ctx->cfg.minibatch) return fail(EMAGPIE_E_ARG, "b must be in [1, minibatch]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  EMG_HIP(emg::launch_slot_info(batch_idx_dev, ctx->pos, ctx->cfg.n_pos, ctx->slots, b, s));
  emg::StepArgs a = base_args(ctx, const_cast<void*>(obj_dev), const_cast<void*>(probe_dev));
  a.slot = ctx->slots;
  a.b = b;
  a.phi = nullptr;
  a.zplus = static_cast<float2*>(zplus_dev);
  a.phase_write = 0;  // a diagnostic: reads the phase memory, leaves it as it was
  EMG_HIP(emg::launch_patch_step(ctx->cfg.m, ctx->cfg.fft_plan, ctx->cfg.levels, a, s));
  return EMAGPIE_OK;
}

emagpie_status emagpie_check_step(emagpie_ctx ctx, void* obj_dev, void* probe_dev,
                                  const int32_t* batch_idx_dev, int32_t b, double* out3_dev,
                                  void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!obj_dev || !probe_dev || !batch_idx_dev || !out3_dev)
    return fail(EMAGPIE_E_ARG, "null argument");
  if (b < 1 || b > ctx->cfg.minibatch) return fail(EMAGPIE_E_ARG, "b must be in [1, minibatch]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int m = ctx->cfg.m, v = ctx->cfg.fft_plan;
  EMG_HIP(emg::launch_slot_info(batch_idx_dev, ctx->pos, ctx->cfg.n_pos, ctx->slots, b, s));
  if (m == 256) {
    emg::StepArgs a = base_args(ctx, obj_dev, probe_dev);
    a.slot = ctx->slots;
    a.b = b;
    EMG_HIP(emg::launch_zero_doubles(out3_dev, 3, s));
    EMG_HIP(emg::launch_check256(a, ctx->cfg.levels, ctx->cfg.finalize_shape, out3_dev, s));
    return EMAGPIE_OK;
  }
  emg::StepArgs a = base_args(ctx, obj_dev, probe_dev);
  a.slot = ctx->slots;
  a.b = b;
  a.sampled = out3_dev;  // [0] accumulates sum_k Phi_k at the state before the step
  EMG_HIP(emg::launch_zero_doubles(out3_dev, 3, s));
  // revised waves R_k frozen at the current iterate (kept in the stack buffer), the step
  EMG_HIP(emg::launch_revised_waves(m, v, a, s));
  EMG_HIP(emg::launch_numerators(m, v, ctx->cfg.levels, a, s));
  EMG_HIP(emg::launch_finalize(m, ctx->cfg.finalize_shape, a, s));
  // [1] surrogate of Eq. 3 at the new state against the frozen R_k, [2] Phi_B at the new state
  EMG_HIP(emg::launch_surrogate_terms(m, v, a, ctx->phi, s));
  EMG_HIP(emg::launch_sum_doubles(ctx->phi, b, out3_dev + 1, s));
  EMG_HIP(emg::launch_misfit_terms(m, v, static_cast<const float2*>(obj_dev), ctx->cfg.n_cols,
                                   static_cast<const float2*>(probe_dev), ctx->dperm, ctx->pos,
                                   ctx->slots, b, ctx->tw32, ctx->phi, 0, s));
  EMG_HIP(emg::launch_sum_doubles(ctx->phi, b, out3_dev + 2, s));
  return EMAGPIE_OK;
}

emagpie_status emagpie_misfit(emagpie_ctx ctx, const void* obj_dev, const void* probe_dev,
                              double* misfit_dev, void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!obj_dev || !probe_dev || !misfit_dev) return fail(EMAGPIE_E_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->cfg.m == 256) {
    // strips and column blocks over the stack buffer, minibatch-sized chunks of patterns
    const emg::StepArgs a = base_args(ctx, const_cast<void*>(obj_dev), const_cast<void*>(probe_dev));
    for (int k0 = 0; k0 < ctx->cfg.n_pos; k0 += ctx->cfg.minibatch) {
      const int cnt = std::min(ctx->cfg.minibatch, ctx->cfg.n_pos - k0);
      EMG_HIP(emg::launch_misfit_strips(256, a, k0, cnt, ctx->phi_all + k0, s));
    }
    EMG_HIP(emg::launch_sum_doubles(ctx->phi_all, ctx->cfg.n_pos, misfit_dev, s));
    return EMAGPIE_OK;
  }
  // the patterns in the context's XCD order, each term at its pattern's index, so the
  // sum runs in pattern order whatever the device
  EMG_HIP(emg::launch_misfit_terms(ctx->cfg.m, ctx->cfg.fft_plan, static_cast<const float2*>(obj_dev),
                                   ctx->cfg.n_cols, static_cast<const float2*>(probe_dev), ctx->dperm,
                                   ctx->pos, ctx->morder, ctx->cfg.n_pos, ctx->tw32, ctx->phi_all, 1, s));
  EMG_HIP(emg::launch_sum_doubles(ctx->phi_all, ctx->cfg.n_pos, misfit_dev, s));
  return EMAGPIE_OK;
}

emagpie_status emagpie_grad(emagpie_ctx ctx, const void* obj_dev, const void* probe_dev,
                            void* grad_obj_dev, void* grad_probe_dev, double* misfit_dev,
                            int32_t dtype, void* stream) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  if (!obj_dev || !probe_dev || !grad_obj_dev || !grad_probe_dev)
    return fail(EMAGPIE_E_ARG, "null argument");
  if (dtype != EMAGPIE_F32 && dtype != EMAGPIE_F64) return fail(EMAGPIE_E_ARG, "dtype must be F32 or F64");
  const bool f64 = dtype == EMAGPIE_F64;
  if (f64 && ctx->cfg.m > 64) return fail(EMAGPIE_E_UNSUPPORTED, "float64 gradient needs m <= 64");
  hipStream_t s = static_cast<hipStream_t>(stream);
  emg::GradArgs g{};
  g.obj = obj_dev;
  g.n = ctx->cfg.n_cols;
  g.nr = ctx->cfg.n_rows;
  g.probe = probe_dev;
  g.dperm = ctx->dperm;
  g.pos = ctx->pos;
  g.n_pos = ctx->cfg.n_pos;
  g.chunk = ctx->lay.grad_chunk;
  g.tw = f64 ? static_cast<const void*>(ctx->tw64) : static_cast<const void*>(ctx->tw32);
  g.gobj = grad_obj_dev;
  g.gprobe = grad_probe_dev;
  g.gz_slots = ctx->ws + ctx->lay.gz.off;
  g.gq_slots = ctx->ws + ctx->lay.gq.off;
  g.phi_all = ctx->phi_all;
  if (ctx->cfg.m == 256) {
    const emg::StepArgs a = base_args(ctx, const_cast<void*>(obj_dev), const_cast<void*>(probe_dev));
    EMG_HIP(emg::launch_grad256(a, g, s));
  } else {
    EMG_HIP(emg::launch_grad(ctx->cfg.m, ctx->cfg.fft_plan, f64, g, s));
  }
  if (misfit_dev) EMG_HIP(emg::launch_sum_doubles(ctx->phi_all, ctx->cfg.n_pos, misfit_dev, s));
  return EMAGPIE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// groups of independent reconstructions
// ---------------------------------------------------------------------------
namespace {

struct GroupClass {
  int m, L, v, f;  // probe side, levels, FFT plan, finalize shape
  std::vector<int> inst;
  std::vector<size_t> patch_off, fin_off;  // per step: offset into the work arrays
  std::vector<int> patch_n, fin_n;         // per step: blocks
};

struct GroupLayout {
  size_t args, slots, work, total;
  int steps;
  std::vector<size_t> slot_off;
  std::vector<GroupClass> classes;
  std::vector<int2> work_host;  // all work lists, concatenated
};

// Per-step work lists of a group of configurations (each resolved, or with
// finalize_shape = EMAGPIE_TUNE when only the size is wanted: the shape with the
// most work items then stands in, so the size is an upper bound).
emagpie_status plan_group_cfgs(const std::vector<emagpie_config>& cfgs, GroupLayout* G) {
  const int n_inst = (int)cfgs.size();
  if (n_inst < 1) return fail(EMAGPIE_E_ARG, "a group needs at least one instance");
  G->steps = 0;
  G->slot_off.assign(n_inst, 0);
  size_t nslots = 0;
  for (int i = 0; i < n_inst; ++i) {
    const emagpie_config& c = cfgs[i];
    if (c.m == 256) return fail(EMAGPIE_E_UNSUPPORTED, "group members need m <= 128");
    G->slot_off[i] = nslots;
    nslots += (size_t)c.n_pos;
    G->steps = std::max(G->steps, (c.n_pos + c.minibatch - 1) / c.minibatch);
  }
  G->classes.clear();
  for (int i = 0; i < n_inst; ++i) {
    const emagpie_config& c = cfgs[i];
    GroupClass* cls = nullptr;
    for (auto& k : G->classes)
      if (k.m == c.m && k.L == c.levels && k.v == c.fft_plan && k.f == c.finalize_shape) cls = &k;
    if (!cls) {
      G->classes.push_back(GroupClass{c.m, c.levels, c.fft_plan, c.finalize_shape, {}, {}, {}, {}, {}});
      cls = &G->classes.back();
    }
    cls->inst.push_back(i);
  }
  G->work_host.clear();
  for (auto& k : G->classes) {
    for (int j = 0; j < G->steps; ++j) {
      k.patch_off.push_back(G->work_host.size());
      for (int i : k.inst) {
        const emagpie_config& c = cfgs[i];
        const int b = std::min(c.minibatch, c.n_pos - j * c.minibatch);
        for (int s = 0; s < b; ++s) G->work_host.push_back(make_int2(j * n_inst + i, s));
      }
      k.patch_n.push_back((int)(G->work_host.size() - k.patch_off.back()));
      k.fin_off.push_back(G->work_host.size());
      for (int i : k.inst) {
        const emagpie_config& c = cfgs[i];
        if (j * c.minibatch >= c.n_pos) continue;
        int items = 0;
        for (int f = 0; f < emg::kFinShapes; ++f) {
          if (c.finalize_shape != EMAGPIE_TUNE && f != c.finalize_shape) continue;
          int it = 0;
          if (emg::finalize_item_count(c.m, f, c.n_rows, c.n_cols, emg::probe_groups(c.minibatch),
                                       &it) != hipSuccess)
            return fail(EMAGPIE_E_SHAPE, "unsupported probe size in group");
          items = std::max(items, it);
        }
        for (int t = 0; t < items; ++t) G->work_host.push_back(make_int2(j * n_inst + i, t));
      }
      k.fin_n.push_back((int)(G->work_host.size() - k.fin_off.back()));
    }
  }
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t o = cur;
    cur += align256(bytes);
    return o;
  };
  G->args = take((size_t)G->steps * n_inst * sizeof(emg::StepArgs));
  G->slots = take(nslots * sizeof(int4));
  G->work = take(G->work_host.size() * sizeof(int2));
  G->total = cur;
  return EMAGPIE_OK;
}

emagpie_status plan_group(int32_t n_inst, const emagpie_ctx* ctxs, GroupLayout* G) {
  if (n_inst < 1 || !ctxs) return fail(EMAGPIE_E_ARG, "a group needs at least one context");
  std::vector<emagpie_config> cfgs(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    if (!ctxs[i]) return fail(EMAGPIE_E_ARG, "null context in group");
    if (ctxs[i]->many) return fail(EMAGPIE_E_ARG, "a many-context cannot be a group member");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(EMAGPIE_E_ARG, "a context appears twice in the group");
    cfgs[i] = ctxs[i]->cfg;
  }
  return plan_group_cfgs(cfgs, G);
}

}  // namespace

struct emagpie_group_s {
  int n;
  std::vector<emagpie_ctx> ctx;
  GroupLayout lay;
  uint8_t* ws = nullptr;
  emg::StepArgs* args_dev = nullptr;
  int4* slots_dev = nullptr;
  int2* work_dev = nullptr;
  std::vector<emg::StepArgs> args_host;
  std::vector<void*> a_obj, a_probe;  // pointers the argument table was built for
  double* a_sampled = nullptr;
  bool args_valid = false;
  std::vector<int32_t> perm_host;
  int4* pinned[2] = {nullptr, nullptr};
  hipEvent_t pin_ev[2] = {nullptr, nullptr};
  int pin_slot = 0;
  std::vector<hipStream_t> streams;  // [0] capture origin, [1..] one per class
  std::vector<hipEvent_t> fork_join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

extern "C" {

emagpie_status emagpie_group_workspace_size(int32_t n_inst, const emagpie_ctx* ctxs, size_t* bytes) {
  if (!bytes) return fail(EMAGPIE_E_ARG, "null output");
  GroupLayout G;
  emagpie_status st = plan_group(n_inst, ctxs, &G);
  if (st != EMAGPIE_OK) return st;
  *bytes = G.total;
  return EMAGPIE_OK;
}

emagpie_status emagpie_group_destroy(emagpie_group g) {
  if (!g) return EMAGPIE_OK;
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (hipEvent_t e : g->fork_join) (void)hipEventDestroy(e);
  for (hipStream_t s : g->streams) (void)hipStreamDestroy(s);
  for (int i = 0; i < 2; ++i) {
    if (g->pin_ev[i]) {
      (void)hipEventSynchronize(g->pin_ev[i]);
      (void)hipEventDestroy(g->pin_ev[i]);
    }
    if (g->pinned[i]) (void)hipHostFree(g->pinned[i]);
  }
  delete g;
  return EMAGPIE_OK;
}

emagpie_status emagpie_group_create(emagpie_group* out, int32_t n_inst, const emagpie_ctx* ctxs,
                                    void* workspace_dev, size_t workspace_bytes, void* stream) {
  if (!out) return fail(EMAGPIE_E_ARG, "null group output");
  *out = nullptr;
  GroupLayout G;
  emagpie_status st = plan_group(n_inst, ctxs, &G);
  if (st != EMAGPIE_OK) return st;
  if (!workspace_dev || (reinterpret_cast<uintptr_t>(workspace_dev) & 255))
    return fail(EMAGPIE_E_WORKSPACE, "group workspace missing or not 256-byte aligned");
  if (workspace_bytes < G.total)
    return fail(EMAGPIE_E_WORKSPACE, "group workspace too small: need " + std::to_string(G.total) +
                                         " bytes, got " + std::to_string(workspace_bytes));
  auto* g = new emagpie_group_s();
  g->n = n_inst;
  g->ctx.assign(ctxs, ctxs + n_inst);
  g->lay = G;
  g->ws = static_cast<uint8_t*>(workspace_dev);
  g->args_dev = reinterpret_cast<emg::StepArgs*>(g->ws + G.args);
  g->slots_dev = reinterpret_cast<int4*>(g->ws + G.slots);
  g->work_dev = reinterpret_cast<int2*>(g->ws + G.work);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto bad = [&](hipError_t e, const char* what) {
    fail(EMAGPIE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    emagpie_group_destroy(g);
    return EMAGPIE_E_HIP;
  };
  hipError_t e;
  if (!G.work_host.empty() &&
      (e = hipMemcpyAsync(g->work_dev, G.work_host.data(), G.work_host.size() * sizeof(int2),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return bad(e, "upload work lists");
  size_t nslots = 0;
  for (auto c : g->ctx) nslots += (size_t)c->cfg.n_pos;
  for (int i = 0; i < 2; ++i) {
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&g->pinned[i]), sizeof(int4) * nslots,
                           hipHostMallocDefault)) != hipSuccess)
      return bad(e, "pinned scan-order buffer");
    if ((e = hipEventCreateWithFlags(&g->pin_ev[i], hipEventDisableTiming)) != hipSuccess)
      return bad(e, "event");
  }
  g->streams.resize(1 + G.classes.size());
  for (auto& st2 : g->streams)
    if ((e = hipStreamCreateWithFlags(&st2, hipStreamNonBlocking)) != hipSuccess)
      return bad(e, "capture stream");
  g->fork_join.resize(1 + G.classes.size());
  for (auto& ev : g->fork_join)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return bad(e, "event");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "synchronise");
  *out = g;
  return EMAGPIE_OK;
}

emagpie_status emagpie_group_epoch(emagpie_group g, void* const* obj_devs, void* const* probe_devs,
                                   int64_t epoch, double* sampled_misfit_dev, void* stream) {
  if (!g || !obj_devs || !probe_devs) return fail(EMAGPIE_E_ARG, "null argument");
  for (int i = 0; i < g->n; ++i)
    if (!obj_devs[i] || !probe_devs[i]) return fail(EMAGPIE_E_ARG, "null object or probe in group");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = g->n, J = g->lay.steps;
  // argument records (rebuilt only when the state buffers change)
  bool same = g->args_valid && g->a_sampled == sampled_misfit_dev;
  for (int i = 0; same && i < n; ++i) same = g->a_obj[i] == obj_devs[i] && g->a_probe[i] == probe_devs[i];
  if (!same) {
    g->args_host.assign((size_t)J * n, emg::StepArgs{});
    for (int j = 0; j < J; ++j)
      for (int i = 0; i < n; ++i) {
        emagpie_ctx c = g->ctx[i];
        emg::StepArgs a = base_args(c, obj_devs[i], probe_devs[i]);
        const int B = c->cfg.minibatch, N = c->cfg.n_pos;
        a.slot = g->slots_dev + g->lay.slot_off[i] + (size_t)std::min(j * B, N);
        a.b = std::max(0, std::min(B, N - j * B));
        a.sampled = sampled_misfit_dev ? sampled_misfit_dev + i : nullptr;
        g->args_host[(size_t)j * n + i] = a;
      }
    EMG_HIP(hipMemcpyAsync(g->args_dev, g->args_host.data(), g->args_host.size() * sizeof(emg::StepArgs),
                           hipMemcpyHostToDevice, s));
    g->a_obj.assign(obj_devs, obj_devs + n);
    g->a_probe.assign(probe_devs, probe_devs + n);
    g->a_sampled = sampled_misfit_dev;
    g->args_valid = true;
  }
  // scan orders of every instance for this epoch, one upload
  const int ps = g->pin_slot;
  g->pin_slot ^= 1;
  EMG_HIP(hipEventSynchronize(g->pin_ev[ps]));
  int4* dst = g->pinned[ps];
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    emagpie_ctx c = g->ctx[i];
    const int N = c->cfg.n_pos;
    g->perm_host.resize(N);
    fisher_yates(c->cfg.seed, epoch, N, g->perm_host.data());
    int4* d = dst + g->lay.slot_off[i];
    for (int j = 0; j < N; ++j) {
      const int k = g->perm_host[j];
      d[j] = make_int4(k, c->pos_host[2 * k], c->pos_host[2 * k + 1], 0);
    }
    xcd_listing_sweep(d, N, std::min(c->cfg.minibatch, N), c->num_xcc, c->listing_tmp);
    total += N;
  }
  EMG_HIP(hipMemcpyAsync(g->slots_dev, dst, total * sizeof(int4), hipMemcpyHostToDevice, s));
  EMG_HIP(hipEventRecord(g->pin_ev[ps], s));
  if (sampled_misfit_dev) EMG_HIP(emg::launch_zero_doubles(sampled_misfit_dev, n, s));
  if (!g->gexec) {
    // capture once: one chain of (patch, finalize) launches per probe-size class,
    // the chains as parallel branches between a fork and a join
    hipStream_t s0 = g->streams[0];
    EMG_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipEventRecord(g->fork_join[0], s0);
    for (size_t c = 0; ce == hipSuccess && c < g->lay.classes.size(); ++c) {
      const GroupClass& k = g->lay.classes[c];
      hipStream_t sc = g->streams[1 + c];
      ce = hipStreamWaitEvent(sc, g->fork_join[0], 0);
      for (int j = 0; ce == hipSuccess && j < J; ++j) {
        if (k.patch_n[j] > 0)
          ce = emg::launch_patch_step_multi(k.m, k.v, k.L, g->args_dev, g->work_dev + k.patch_off[j],
                                            k.patch_n[j], sc);
        if (ce == hipSuccess && k.fin_n[j] > 0)
          ce = emg::launch_finalize_multi(k.m, k.f, g->args_dev, g->work_dev + k.fin_off[j], k.fin_n[j],
                                          sc);
      }
      if (ce == hipSuccess) ce = hipEventRecord(g->fork_join[1 + c], sc);
      if (ce == hipSuccess) ce = hipStreamWaitEvent(s0, g->fork_join[1 + c], 0);
    }
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(s0, &graph);
    if (ce != hipSuccess || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(EMAGPIE_E_HIP, std::string("group capture: ") +
                                     hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    g->graph = graph;
    EMG_HIP(hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0));
  }
  EMG_HIP(hipGraphLaunch(g->gexec, s));
  return EMAGPIE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// many instances behind one context, fault injection, measured peaks
// ---------------------------------------------------------------------------
struct Many {
  std::vector<emagpie_ctx> members;
  emagpie_group group = nullptr;
};

namespace {

// member workspaces (256-byte aligned, in order), then the group workspace
struct ManyLayout {
  std::vector<size_t> off, bytes;
  size_t group_off = 0, group_bytes = 0, total = 0;
};

emagpie_status many_layout(int32_t n_inst, const emagpie_config* cfgs, ManyLayout* M) {
  if (n_inst < 1 || !cfgs) return fail(EMAGPIE_E_ARG, "emagpie_init_many needs at least one configuration");
  size_t cur = 0;
  std::vector<emagpie_config> v(cfgs, cfgs + n_inst);
  for (int i = 0; i < n_inst; ++i) {
    emagpie_status st = check_config(&cfgs[i]);
    if (st != EMAGPIE_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_err);
    const size_t b = make_layout(cfgs[i]).total;
    M->off.push_back(cur);
    M->bytes.push_back(b);
    cur += align256(b);
  }
  GroupLayout G;
  EMG_OK(plan_group_cfgs(v, &G));
  M->group_off = cur;
  M->group_bytes = G.total;
  M->total = cur + align256(G.total);
  return EMAGPIE_OK;
}

}  // namespace

void destroy_many(emagpie_ctx ctx) {
  Many* mm = ctx->many;
  if (mm->group) (void)emagpie_group_destroy(mm->group);
  for (emagpie_ctx c : mm->members) (void)emagpie_destroy(c);
  delete mm;
  delete ctx;
}

extern "C" {

emagpie_status emagpie_workspace_size_many(int32_t n_inst, const emagpie_config* cfgs, size_t* bytes) {
  if (!bytes) return fail(EMAGPIE_E_ARG, "null output");
  ManyLayout M;
  EMG_OK(many_layout(n_inst, cfgs, &M));
  *bytes = M.total;
  return EMAGPIE_OK;
}

emagpie_status emagpie_init_many(emagpie_ctx* out, int32_t n_inst, const emagpie_config* cfgs,
                                 const int32_t* const* positions_host,
                                 const float* const* intensities_dev, void* workspace_dev,
                                 size_t workspace_bytes, void* stream) {
  if (!out) return fail(EMAGPIE_E_ARG, "null context output");
  *out = nullptr;
  if (!positions_host || !intensities_dev) return fail(EMAGPIE_E_ARG, "null positions or intensities array");
  ManyLayout M;
  EMG_OK(many_layout(n_inst, cfgs, &M));
  if (!workspace_dev || (reinterpret_cast<uintptr_t>(workspace_dev) & 255))
    return fail(EMAGPIE_E_WORKSPACE, "workspace missing or not 256-byte aligned");
  if (workspace_bytes < M.total)
    return fail(EMAGPIE_E_WORKSPACE, "workspace too small: need " + std::to_string(M.total) +
                                         " bytes, got " + std::to_string(workspace_bytes));
  uint8_t* w = static_cast<uint8_t*>(workspace_dev);
  auto* mm = new Many();
  auto* ctx = new emagpie_ctx_s();
  ctx->cfg = cfgs[0];
  ctx->many = mm;
  for (int i = 0; i < n_inst; ++i) {
    emagpie_ctx c = nullptr;
    emagpie_status st = emagpie_init(&c, &cfgs[i], positions_host[i], intensities_dev[i], w + M.off[i],
                                     M.bytes[i], stream);
    if (st != EMAGPIE_OK) {
      const std::string msg = "instance " + std::to_string(i) + ": " + g_err;
      destroy_many(ctx);
      return fail(st, msg);
    }
    mm->members.push_back(c);
  }
  emagpie_status st = emagpie_group_create(&mm->group, n_inst, mm->members.data(), w + M.group_off,
                                           M.group_bytes, stream);
  if (st != EMAGPIE_OK) {
    const std::string msg = g_err;
    destroy_many(ctx);
    return fail(st, msg);
  }
  *out = ctx;
  return EMAGPIE_OK;
}

emagpie_status emagpie_epoch_many(emagpie_ctx ctx, void* const* obj_devs, void* const* probe_devs,
                                  int64_t epoch, double* sampled_misfit_dev, void* stream) {
  CtxErrScope es_(ctx);
  if (!ctx || !ctx->many) return fail(EMAGPIE_E_ARG, "not a context made by emagpie_init_many");
  for (emagpie_ctx c : ctx->many->members) EMG_OK(use_ctx(c));
  return emagpie_group_epoch(ctx->many->group, obj_devs, probe_devs, epoch, sampled_misfit_dev, stream);
}

emagpie_status emagpie_many_member(emagpie_ctx ctx, int32_t i, emagpie_ctx* member_out) {
  CtxErrScope es_(ctx);
  if (!ctx || !ctx->many || !member_out) return fail(EMAGPIE_E_ARG, "null argument or not a many-context");
  if (i < 0 || i >= (int)ctx->many->members.size()) return fail(EMAGPIE_E_ARG, "member index out of range");
  *member_out = ctx->many->members[i];
  return EMAGPIE_OK;
}

emagpie_status emagpie_debug_barrier(emagpie_ctx ctx, uint32_t spin_limit, uint32_t target_skew) {
  CtxErrScope es_(ctx);
  EMG_OK(use_ctx(ctx));
  ctx->spin_limit = spin_limit ? spin_limit : kDefaultSpinLimit;
  ctx->bar_skew = target_skew;
  return EMAGPIE_OK;
}

emagpie_status emagpie_measure_peaks(void* buf_dev, size_t bytes, int32_t reps, double* out2_host,
                                     void* stream) {
  if (!buf_dev || !out2_host || reps < 1) return fail(EMAGPIE_E_ARG, "null buffer or output, or reps < 1");
  if ((reinterpret_cast<uintptr_t>(buf_dev) & 255) || bytes < (size_t(4) << 20))
    return fail(EMAGPIE_E_WORKSPACE, "buffer must be 256-byte aligned and at least 4 MiB");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  EMG_HIP(hipGetDevice(&dev));
  EMG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const size_t n4 = bytes / 2 / 16;
  uint8_t* b = static_cast<uint8_t*>(buf_dev);
  const int copy_blocks = 16 * cus, fma_blocks = 8 * cus, fma_iters = 4096;
  if ((size_t)fma_blocks * 256 * sizeof(float) > bytes)
    return fail(EMAGPIE_E_WORKSPACE, "buffer too small for the FMA loop's output");
  double flops = 0.0;
  std::vector<float> t_copy, t_fma;
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  emagpie_status st = EMAGPIE_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) st = fail(EMAGPIE_E_HIP, "peak-measurement event");
  for (int pass = 0; st == EMAGPIE_OK && pass < 2; ++pass) {
    // one untimed launch, then reps timed ones
    for (int i = -1; st == EMAGPIE_OK && i < reps; ++i) {
      if (i >= 0 && hipEventRecord(ev[2 * i], s) != hipSuccess) st = fail(EMAGPIE_E_HIP, "event record");
      const hipError_t e = pass == 0 ? emg::launch_copy16(b, b + n4 * 16, n4, copy_blocks, s)
                                     : emg::launch_fma_loop(reinterpret_cast<float*>(b), fma_blocks,
                                                            fma_iters, s, &flops);
      if (e != hipSuccess) st = fail(EMAGPIE_E_HIP, std::string("peak kernel: ") + hipGetErrorString(e));
      if (st == EMAGPIE_OK && i >= 0 && hipEventRecord(ev[2 * i + 1], s) != hipSuccess)
        st = fail(EMAGPIE_E_HIP, "event record");
    }
    if (st == EMAGPIE_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(EMAGPIE_E_HIP, "synchronise");
    for (int i = 0; st == EMAGPIE_OK && i < reps; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) st = fail(EMAGPIE_E_HIP, "timing");
      (pass == 0 ? t_copy : t_fma).push_back(ms);
    }
  }
  (void)hipStreamSynchronize(s);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st != EMAGPIE_OK) return st;
  out2_host[0] = 2.0 * (double)n4 * 16.0 / (median(t_copy) * 1e-3) / 1e9;
  out2_host[1] = flops / (median(t_fma) * 1e-3) / 1e12;
  return EMAGPIE_OK;
}

}  // extern "C"
