// C ABI of the library (declared in include/sht.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "interp_decomp.h"
#include "plan_cache.h"
#include "sht_internal.h"

namespace sht {
int build_plan(sht_plan_s* P, const sht_plan_opts& o);
void free_plan_device(sht_plan_s* P);
}  // namespace sht

using namespace sht;

struct sht_bf_s {
  BfTree tree;
};

namespace sht {

int Profiler::find_or_add(const std::string& name, double flops, double bytes) {
  for (size_t i = 0; i < recs.size(); ++i)
    if (recs[i].name == name) return static_cast<int>(i);
  ProfRecord r;
  r.name = name;
  r.flops = flops;
  r.bytes = bytes;
  recs.push_back(r);
  return static_cast<int>(recs.size()) - 1;
}

int Profiler::flush() {
  int rc = SHT_OK;
  for (auto& p : pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess)
      rc = SHT_EHIP;
    recs[p.rec].ms += ms;
    recs[p.rec].launches += 1;
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  pending.clear();
  return rc;
}

void Profiler::clear() {
  (void)flush();
  recs.clear();
}

hipError_t ensure_split_factors(sht_plan_s* P, hipStream_t s) {
  std::lock_guard<std::mutex> lock(P->split_mu);
  return split_factors(P, s);
}

}  // namespace sht

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Workspace {
  double* xin;
  double* v0;
  double* v1;
  double* y;
};

int field_width(const sht_plan_s* P, int F) { return P->kind == SHT_COMPLEX ? 4 * F : 2 * F; }

size_t ws_bytes(const sht_plan_s* P, int F) {
  const size_t R = static_cast<size_t>(field_width(P, F));
  return align256(P->rows_in * R * 8) + 2 * align256(P->rows_v * R * 8) +
         align256(P->rows_y * R * 8);
}

Workspace carve(const sht_plan_s* P, int F, void* ws) {
  const size_t R = static_cast<size_t>(field_width(P, F));
  char* p = static_cast<char*>(ws);
  Workspace w;
  w.xin = reinterpret_cast<double*>(p);
  p += align256(P->rows_in * R * 8);
  w.v0 = reinterpret_cast<double*>(p);
  p += align256(P->rows_v * R * 8);
  w.v1 = reinterpret_cast<double*>(p);
  p += align256(P->rows_v * R * 8);
  w.y = reinterpret_cast<double*>(p);
  return w;
}

class DeviceScope {
 public:
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev && dev >= 0) {
      ok_ = hipSetDevice(dev) == hipSuccess;
      switched_ = true;
    }
  }
  ~DeviceScope() {
    if (switched_ && prev_ >= 0) (void)hipSetDevice(prev_);
  }
  bool ok() const { return ok_; }

 private:
  int prev_ = -1;
  bool switched_ = false;
  bool ok_ = true;
};

}  // namespace

// ------------------------------------------------------------ allocation and call tracing

namespace sht {

namespace {
// allocations left before the injected failures begin; -1: no injection
std::atomic<long long> g_alloc_left{-1};

bool alloc_refused() {
  long long v = g_alloc_left.load(std::memory_order_relaxed);
  while (v > 0 && !g_alloc_left.compare_exchange_weak(v, v - 1, std::memory_order_relaxed)) {
  }
  return v == 0;
}

double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

hipError_t dev_alloc(void** p, size_t bytes) {
  if (alloc_refused()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

hipError_t pinned_alloc(void** p, size_t bytes) {
  if (alloc_refused()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipHostMalloc(p, bytes);
}

AllocFaultScope::AllocFaultScope() {
  const char* e = std::getenv("SHT_TEST_FAIL_ALLOC_AFTER");
  const long long n = e && *e ? std::atoll(e) : -1;
  g_alloc_left.store(n < 0 ? -1 : n, std::memory_order_relaxed);
}

AllocFaultScope::~AllocFaultScope() { g_alloc_left.store(-1, std::memory_order_relaxed); }

TraceCall::TraceCall(const char* name, int device, void* stream) : name_(name), device_(device), stream_(stream) {
  const char* e = std::getenv("SHT_TRACE");
  level_ = e && *e ? std::atoi(e) : 0;
  if (level_ <= 0) return;
  t0_ = wall_ms();
  if (level_ >= 2 && device_ >= 0) {
    DeviceScope ds(device_);
    if (ds.ok() && hipEventCreate(&ev_[0]) == hipSuccess && hipEventCreate(&ev_[1]) == hipSuccess)
      (void)hipEventRecord(ev_[0], static_cast<hipStream_t>(stream_));
  }
}

TraceCall::~TraceCall() {
  if (!ev_[0] && !ev_[1]) return;
  DeviceScope ds(device_);
  for (hipEvent_t& e : ev_)
    if (e) (void)hipEventDestroy(e);
}

void TraceCall::args(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(args_, sizeof(args_), fmt, ap);
  va_end(ap);
}

int TraceCall::done(int rc) {
  if (level_ <= 0) return rc;
  const double host_ms = wall_ms() - t0_;
  char dev[48] = "";
  if (ev_[0] && ev_[1]) {
    DeviceScope ds(device_);
    float ms = 0.0f;
    if (hipEventRecord(ev_[1], static_cast<hipStream_t>(stream_)) == hipSuccess &&
        hipEventSynchronize(ev_[1]) == hipSuccess && hipEventElapsedTime(&ms, ev_[0], ev_[1]) == hipSuccess)
      std::snprintf(dev, sizeof(dev), ", device %.3f ms", static_cast<double>(ms));
  }
  std::fprintf(stderr, "sht: %s(%s) -> %d (%s), host %.3f ms%s\n", name_, args_, rc, sht_strerror(rc), host_ms,
               dev);
  return rc;
}

}  // namespace sht

namespace {

int check_call(const sht_plan_s* P, int precision, const void* a, const void* b, int F, void* ws,
               size_t wsb) {
  if (!P || !a || !b || F < 1 || !ws) return SHT_EINVAL;
  if (P->maps) return SHT_EINVAL;  // a plan of the per-order maps has no SHT
  if (precision < SHT_FP64 || precision > SHT_INT8) return SHT_EINVAL;
  // the split, FP32 and int8 forms run on the matrix-core kernels only (R a multiple of 16),
  // on factor copies that sht_plan_prepare (or a plan built for that precision) derived
  if (precision != SHT_FP64 && !mfma_ok(field_width(P, F))) return SHT_EUNSUPPORTED;
  if ((precision == SHT_SPLIT32 || precision == SHT_FP32) && !P->d.fac_hl) return SHT_ENOTREADY;
  if (precision == SHT_INT8 && !P->d.dig) return SHT_ENOTREADY;
  if (precision == SHT_FP64 && !P->d.fac) return SHT_ENOTREADY;  // a split-only plan
  if (reinterpret_cast<uintptr_t>(a) % 16 || reinterpret_cast<uintptr_t>(b) % 16) return SHT_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return SHT_EINVAL;
  if (wsb < ws_bytes(P, F)) return SHT_EINVAL;
  if (static_cast<long long>(field_width(P, F)) * std::max(P->rows_y, P->rows_in) > (1LL << 40))
    return SHT_EUNSUPPORTED;
  return SHT_OK;
}

#define HIP_OK(expr)                          \
  do {                                        \
    if ((expr) != hipSuccess) return SHT_EHIP; \
  } while (0)

// Algorithmic work of each stage for F fields (flops, HBM bytes per launch).
struct Work {
  double flops, bytes;
};

Work level_work(const sht_plan_s* P, int t, int R) {
  return {2.0 * P->step_fac[t] * R,
          8.0 * (P->step_fac[t] + (P->step_rows_in[t] + P->step_rows_out[t]) * R)};
}
Work final_work(const sht_plan_s* P, int R) {
  return {2.0 * P->final_fac * R, 8.0 * (P->final_fac + (P->final_rows_v + P->final_rows_y) * R)};
}
Work class_work(const LaunchClass& c, int R) {
  return {2.0 * c.fac * R, 8.0 * (c.fac + (c.rows_in + c.rows_out) * R)};
}
Work fft_work(const sht_plan_s* P, int F, int R) {
  const double N = 4.0 * P->l;
  const double rows = 2.0 * P->l * F;
  const double grid_word = P->kind == SHT_COMPLEX ? 16.0 : 8.0;
  return {5.0 * N * std::log2(N) * rows, 8.0 * P->rows_y * R + rows * N * grid_word};
}
Work layout_work(const sht_plan_s* P, int F, int R) {
  const double ncoef = P->kind == SHT_COMPLEX ? 4.0 * P->l * P->l : 2.0 * P->l * P->l + P->l;
  return {0.0, 16.0 * ncoef * F + 8.0 * P->rows_in * R};
}

// Runs one launch; with profiling on (prof), brackets it with events on the stream.  The
// stage name and work are evaluated only then, so an unprofiled call builds no strings.
template <typename Name, typename Fn>
int stage(sht_plan_s* P, hipStream_t s, bool prof, Name&& name, Fn&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  int rec = -1;
  auto fail = [&]() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return SHT_EHIP;
  };
  if (prof) {
    const std::pair<std::string, Work> nw = name();
    rec = P->prof.find_or_add(nw.first, nw.second.flops, nw.second.bytes);
    if (hipEventCreate(&a) != hipSuccess || hipEventRecord(a, s) != hipSuccess) return fail();
  }
  if (launch() != hipSuccess) return fail();
  if (prof) {
    if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s) != hipSuccess) return fail();
    P->prof.pending.push_back({rec, a, b});
  }
  return SHT_OK;
}

// `prof` (bool) must be in scope: profiling wanted for this call.
#define STAGE(name, work, call)                                                          \
  do {                                                                                   \
    int _rc = stage(P, s, prof, [&]() { return std::pair<std::string, Work>((name), (work)); }, \
                    [&]() { return (call); });                                           \
    if (_rc != SHT_OK) return _rc;                                                       \
  } while (0)

std::string fsuffix(int F, int precision) {
  const char* tag = precision == SHT_SPLIT32 ? "/split32"
                    : precision == SHT_FP32  ? "/fp32"
                    : precision == SHT_INT8  ? "/int8"
                                             : "/fp64";
  return "/F" + std::to_string(F) + tag;
}

}  // namespace

namespace sht {

// Synthesis into the caller's workspace; allow_prof = false runs without the per-stage events
// even when the plan's profiler is on (no event objects, no strings: nothing is allocated).
int run_synth(sht_plan_s* P, int precision, const double* coeff, double* grid, int F, void* ws,
              size_t wsb, void* stream, bool allow_prof) {
  int rc = check_call(P, precision, coeff, grid, F, ws, wsb);
  if (rc) return rc;
  DeviceScope ds(P->device);
  if (!ds.ok()) return SHT_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int R = field_width(P, F);
  Workspace w = carve(P, F, ws);
  const bool prof = allow_prof && P->prof.on;
  const std::string fs = prof ? fsuffix(F, precision) : std::string();
  // matrix-core path: one stage per size-class launch ("synth.level2.c1/F64/fp64"), so that every
  // timed stage is exactly one kernel dispatch; the leaf kernels gather straight from the
  // coefficient layout
  const bool mf = mfma_ok(R);
  if (mf) {
    for (size_t c = 0; c < P->step_classes[0].size(); ++c)
      STAGE("synth.level0.c" + std::to_string(c) + fs, class_work(P->step_classes[0][c], R),
            launch_level(P, 0, false, nullptr, w.v0, R, precision, s, const_cast<double*>(coeff),
                         static_cast<int>(c)));
  } else {
    STAGE("synth.layout" + fs, layout_work(P, F, R), launch_coeff_to_xin(P, coeff, w.xin, F, R, s));
    if (P->step_cnt[0] > 0)
      STAGE("synth.level0" + fs, level_work(P, 0, R),
            launch_level(P, 0, false, w.xin, w.v0, R, precision, s, nullptr, -1, w.xin));
  }
  for (int t = 1; t <= P->Lmax; ++t) {
    const double* in = (t - 1) % 2 ? w.v1 : w.v0;
    double* out = t % 2 ? w.v1 : w.v0;
    if (mf) {
      for (size_t c = 0; c < P->step_classes[t].size(); ++c)
        STAGE("synth.level" + std::to_string(t) + ".c" + std::to_string(c) + fs,
              class_work(P->step_classes[t][c], R),
              launch_level(P, t, false, in, out, R, precision, s, const_cast<double*>(coeff),
                           static_cast<int>(c)));
    } else {
      STAGE("synth.level" + std::to_string(t) + fs, level_work(P, t, R),
            launch_level(P, t, false, in, out, R, precision, s, nullptr, -1, w.xin));
    }
  }
  if (mf) {
    for (size_t c = 0; c < P->final_classes.size(); ++c)
      STAGE("synth.final.c" + std::to_string(c) + fs, class_work(P->final_classes[c], R),
            launch_final(P, false, w.v0, w.v1, nullptr, nullptr, w.y, nullptr, R, precision, false, s,
                         static_cast<int>(c)));
  } else {
    STAGE("synth.final" + fs, final_work(P, R),
          launch_final(P, false, w.v0, w.v1, nullptr, nullptr, w.y, nullptr, R, precision, false, s));
  }
  STAGE("synth.fft" + fs, fft_work(P, F, R), launch_fft_synth(P, w.y, grid, F, R, s));
  return SHT_OK;
}

size_t synth_workspace_bytes(const sht_plan_s* P, int F) { return ws_bytes(P, F); }

}  // namespace sht

namespace {

int run_transposed(sht_plan_s* P, int precision, const double* grid, double* coeff, int F, void* ws,
                   size_t wsb, void* stream, bool adjoint) {
  int rc = check_call(P, precision, grid, coeff, F, ws, wsb);
  if (rc) return rc;
  DeviceScope ds(P->device);
  if (!ds.ok()) return SHT_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int R = field_width(P, F);
  Workspace w = carve(P, F, ws);
  const double scale = adjoint ? 1.0 : 1.0 / (4.0 * P->l);
  const bool prof = P->prof.on;
  const std::string pre = adjoint ? "adjoint." : "analysis.";
  const std::string fs = prof ? fsuffix(F, precision) : std::string();
  STAGE(pre + "fft" + fs, fft_work(P, F, R),
        launch_fft_analyze(P, grid, w.y, F, R, scale, adjoint ? 2.0 : 1.0, s));
  STAGE(pre + "final" + fs, final_work(P, R),
        launch_final(P, true, nullptr, nullptr, w.v0, w.v1, nullptr, w.y, R, precision, adjoint, s));
  const bool mf = mfma_ok(R);
  for (int t = P->Lmax; t >= 1; --t) {
    const double* in = t % 2 ? w.v1 : w.v0;
    double* out = (t - 1) % 2 ? w.v1 : w.v0;
    if (mf) {
      for (size_t c = 0; c < P->step_classes[t].size(); ++c)
        STAGE(pre + "level" + std::to_string(t) + ".c" + std::to_string(c) + fs,
              class_work(P->step_classes[t][c], R),
              launch_level(P, t, true, in, out, R, precision, s, coeff, static_cast<int>(c)));
    } else {
      STAGE(pre + "level" + std::to_string(t) + fs, level_work(P, t, R),
            launch_level(P, t, true, in, out, R, precision, s, nullptr, -1, w.xin));
    }
  }
  if (mf) {  // the transposed leaf kernels scatter straight into the coefficient layout
    for (size_t c = 0; c < P->step_classes[0].size(); ++c)
      STAGE(pre + "level0.c" + std::to_string(c) + fs, class_work(P->step_classes[0][c], R),
            launch_level(P, 0, true, w.v0, nullptr, R, precision, s, coeff, static_cast<int>(c)));
  } else {
    if (P->step_cnt[0] > 0)
      STAGE(pre + "level0" + fs, level_work(P, 0, R),
            launch_level(P, 0, true, w.v0, w.xin, R, precision, s, nullptr, -1, w.xin));
    STAGE(pre + "layout" + fs, layout_work(P, F, R), launch_xin_to_coeff(P, w.xin, coeff, F, R, s));
  }
  return SHT_OK;
}

}  // namespace

extern "C" {

void sht_default_opts(sht_plan_opts* o) {
  if (!o) return;
  o->leaf_width = 64;
  o->precision = SHT_FP64;
  o->field_kind = SHT_COMPLEX;
  o->host_threads = 0;
  o->device = -1;
  o->split_only = 0;
  o->cache_dir = nullptr;
  o->id_device = 0;
}

int sht_plan(int l, double eps, sht_plan_t* out) { return sht_plan_ex(l, eps, nullptr, out); }

namespace {

// Builds and uploads a plan (validated options); maps: the per-order maps of Section 5.
int make_plan(int l, double eps, const sht_plan_opts& o, bool maps, sht_plan_t* out) {
  int dev = o.device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return SHT_EHIP;
  DeviceScope ds(dev);
  if (!ds.ok()) return SHT_EHIP;
  AllocFaultScope faults;
  sht_plan_s* P = new (std::nothrow) sht_plan_s();
  if (!P) return SHT_ENOMEM;
  P->l = l;
  P->C = o.leaf_width;
  P->eps = eps;
  P->device = dev;
  P->precision = o.precision;
  P->kind = o.field_kind;
  P->maps = maps;
  int rc;
  try {
    rc = build_plan(P, o);
  } catch (const std::bad_alloc&) {
    rc = SHT_ENOMEM;
  } catch (...) {
    rc = SHT_EINTERNAL;
  }
  // a plan built for a split, FP32 or int8 default derives those factor copies now, so that
  // its transforms never allocate or wait
  if (rc == SHT_OK && P->precision != SHT_FP64) {
    const hipError_t e = P->precision == SHT_INT8 ? i8_prepare(P, nullptr) : split_factors(P, nullptr);
    if (e != hipSuccess) rc = e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EHIP;
  }
  if (rc == SHT_OK && o.split_only) {
    (void)hipFree(P->d.fac);
    (void)hipFree(P->d.fac_t);
    P->d.fac = P->d.fac_t = nullptr;
    P->stats.device_bytes -= static_cast<long long>(2 * P->n_fac * sizeof(double));
  }
  if (rc != SHT_OK) {
    free_plan_device(P);
    delete P;
    return rc;
  }
  *out = P;
  return SHT_OK;
}

}  // namespace

static int plan_ex(int l, double eps, const sht_plan_opts* opts, sht_plan_t* out) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  sht_plan_opts o;
  sht_default_opts(&o);
  if (opts) o = *opts;
  if (o.leaf_width == 0) o.leaf_width = 64;
  if (l < 1 || !(eps > 0.0 && eps < 1.0) || o.leaf_width < 1 || o.leaf_width > 4096)
    return SHT_EINVAL;
  if (o.precision < SHT_FP64 || o.precision > SHT_INT8) return SHT_EINVAL;
  if (o.field_kind != SHT_COMPLEX && o.field_kind != SHT_REAL) return SHT_EINVAL;
  if (o.split_only && o.precision == SHT_FP64) return SHT_EINVAL;
  if (!pow2(l) || l > 2048) return SHT_EUNSUPPORTED;
  return make_plan(l, eps, o, false, out);
}

int sht_plan_ex(int l, double eps, const sht_plan_opts* opts, sht_plan_t* out) {
  TraceCall tc("sht_plan_ex", -1, nullptr);
  if (tc.on())
    tc.args("l=%d, eps=%g, leaf_width=%d, precision=%d, id_device=%d", l, eps, opts ? opts->leaf_width : 0,
            opts ? opts->precision : SHT_FP64, opts ? opts->id_device : 0);
  return tc.done(plan_ex(l, eps, opts, out));
}

static int order_plan(int l, double eps, const sht_plan_opts* opts, sht_plan_t* out) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  sht_plan_opts o;
  sht_default_opts(&o);
  if (opts) o = *opts;
  if (o.leaf_width == 0) o.leaf_width = 64;
  if (l < 1 || !(eps > 0.0 && eps < 1.0) || o.leaf_width < 2 || o.leaf_width > 4096) return SHT_EINVAL;
  if (o.precision < SHT_FP64 || o.precision > SHT_INT8) return SHT_EINVAL;
  if (l > 2048 || o.precision != SHT_FP64 || o.split_only || o.cache_dir || o.id_device) return SHT_EUNSUPPORTED;
  return make_plan(l, eps, o, true, out);
}

int sht_order_plan(int l, double eps, const sht_plan_opts* opts, sht_plan_t* out) {
  TraceCall tc("sht_order_plan", -1, nullptr);
  if (tc.on()) tc.args("l=%d, eps=%g, leaf_width=%d", l, eps, opts ? opts->leaf_width : 0);
  return tc.done(order_plan(l, eps, opts, out));
}

long long sht_order_rows(sht_plan_t plan) {
  if (!plan || !plan->maps) return SHT_EINVAL;
  return plan->rows_in;
}

int sht_order_layout(sht_plan_t plan, int m, int p, long long* row0, int* n) {
  if (!plan || !plan->maps || m < 0 || m >= 2 * plan->l || (p != 0 && p != 1)) return SHT_EINVAL;
  if (row0) *row0 = plan->in_base[2 * m + p];
  if (n) *n = plan->n_cols[2 * m + p];
  return SHT_OK;
}

size_t sht_order_workspace_bytes(sht_plan_t plan, int R) {
  if (!plan || !plan->maps || R < 1) return 0;
  return 2 * align256(static_cast<size_t>(plan->rows_v) * R * 8);
}

static int order_apply(sht_plan_t plan, const double* in, double* out, int R, int transpose, void* ws, size_t wsb,
                       void* stream) {
  sht_plan_s* P = plan;
  if (!P || !P->maps || !in || !out || !ws || R < 1 || R > 65535 || (transpose != 0 && transpose != 1))
    return SHT_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % 16 || reinterpret_cast<uintptr_t>(out) % 16 ||
      reinterpret_cast<uintptr_t>(ws) % 256)
    return SHT_EINVAL;
  if (wsb < sht_order_workspace_bytes(plan, R)) return SHT_EINVAL;
  const size_t bytes = static_cast<size_t>(P->rows_in) * R * 8;
  const char *a = reinterpret_cast<const char*>(in), *b = reinterpret_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return SHT_EINVAL;  // in and out overlap
  DeviceScope ds(P->device);
  if (!ds.ok()) return SHT_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* v0 = static_cast<double*>(ws);
  double* v1 = reinterpret_cast<double*>(static_cast<char*>(ws) + align256(static_cast<size_t>(P->rows_v) * R * 8));
  const bool prof = P->prof.on;
  const std::string fs = prof ? "/R" + std::to_string(R) + "/fp64" : std::string();
  const Work fw{2.0 * P->final_fac * R, 8.0 * (P->final_fac + (P->final_rows_v + P->final_rows_y) * R)};
  double* xin = const_cast<double*>(in);
  if (!transpose) {
    if (P->step_cnt[0] > 0)
      STAGE("order.level0" + fs, level_work(P, 0, R),
            launch_level(P, 0, false, in, v0, R, SHT_FP64, s, nullptr, -1, xin));
    for (int t = 1; t <= P->Lmax; ++t)
      STAGE("order.level" + std::to_string(t) + fs, level_work(P, t, R),
            launch_level(P, t, false, (t - 1) % 2 ? v1 : v0, t % 2 ? v1 : v0, R, SHT_FP64, s, nullptr, -1, xin));
    STAGE("order.final" + fs, fw, launch_order_final(P, false, v0, v1, nullptr, nullptr, out, nullptr, R, s));
  } else {
    STAGE("order_t.final" + fs, fw, launch_order_final(P, true, nullptr, nullptr, v0, v1, nullptr, in, R, s));
    for (int t = P->Lmax; t >= 1; --t)
      STAGE("order_t.level" + std::to_string(t) + fs, level_work(P, t, R),
            launch_level(P, t, true, t % 2 ? v1 : v0, (t - 1) % 2 ? v1 : v0, R, SHT_FP64, s, nullptr, -1, out));
    if (P->step_cnt[0] > 0)
      STAGE("order_t.level0" + fs, level_work(P, 0, R),
            launch_level(P, 0, true, v0, out, R, SHT_FP64, s, nullptr, -1, out));
  }
  return SHT_OK;
}

int sht_order_apply(sht_plan_t plan, const double* in, double* out, int R, int transpose, void* ws, size_t wsb,
                    void* stream) {
  TraceCall tc("sht_order_apply", plan ? plan->device : -1, stream);
  if (tc.on()) tc.args("l=%d, R=%d, transpose=%d", plan ? plan->l : 0, R, transpose);
  return tc.done(order_apply(plan, in, out, R, transpose, ws, wsb, stream));
}

static int plan_prepare(sht_plan_t plan, int precision, void* stream) {
  if (!plan) return SHT_EINVAL;
  if (precision < SHT_FP64 || precision > SHT_INT8) return SHT_EINVAL;
  if (plan->maps && precision != SHT_FP64) return SHT_EUNSUPPORTED;
  if (precision == SHT_FP64) return plan->d.fac ? SHT_OK : SHT_ENOTREADY;
  DeviceScope ds(plan->device);
  if (!ds.ok()) return SHT_EHIP;
  if (!plan->d.fac && ((precision == SHT_INT8 && !plan->d.dig) || (precision != SHT_INT8 && !plan->d.fac_hl)))
    return SHT_ENOTREADY;  // a split-only plan no longer holds the FP64 factors they come from
  hipError_t e;
  {
    std::lock_guard<std::mutex> lock(plan->split_mu);
    AllocFaultScope faults;
    e = precision == SHT_INT8 ? i8_prepare(plan, static_cast<hipStream_t>(stream))
                              : split_factors(plan, static_cast<hipStream_t>(stream));
  }
  if (e == hipErrorOutOfMemory) return SHT_ENOMEM;
  return e == hipSuccess ? SHT_OK : SHT_EHIP;
}

int sht_plan_prepare(sht_plan_t plan, int precision, void* stream) {
  TraceCall tc("sht_plan_prepare", plan ? plan->device : -1, stream);
  if (tc.on()) tc.args("l=%d, precision=%d", plan ? plan->l : 0, precision);
  return tc.done(plan_prepare(plan, precision, stream));
}

void sht_destroy(sht_plan_t plan) {
  TraceCall tc("sht_destroy", -1, nullptr);
  if (tc.on()) tc.args("l=%d", plan ? plan->l : 0);
  tc.done(SHT_OK);
  if (!plan) return;
  DeviceScope ds(plan->device);
  plan->prof.clear();
  free_plan_device(plan);
  delete plan;
}

size_t sht_workspace_bytes(sht_plan_t plan, int nfields, int precision) {
  if (!plan || plan->maps || nfields < 1 || precision < SHT_FP64 || precision > SHT_INT8) return 0;
  return ws_bytes(plan, nfields);
}

namespace {
// One traced transform call: op 0 synthesis, 1 analysis, 2 adjoint of synthesis.
int traced_transform(const char* name, sht_plan_t plan, int prec, const double* in, double* out, int F, void* ws,
                     size_t wsb, void* stream, int op) {
  TraceCall tc(name, plan ? plan->device : -1, stream);
  if (tc.on()) tc.args("l=%d, F=%d, precision=%d", plan ? plan->l : 0, F, prec);
  if (!plan) return tc.done(SHT_EINVAL);
  if (op == 0) return tc.done(run_synth(plan, prec, in, out, F, ws, wsb, stream, true));
  return tc.done(run_transposed(plan, prec, in, out, F, ws, wsb, stream, op == 2));
}
}  // namespace

int sht_synth(sht_plan_t plan, const double* coeff, double* grid, int F, void* ws, size_t wsb,
              void* stream) {
  return traced_transform("sht_synth", plan, plan ? plan->precision : SHT_FP64, coeff, grid, F, ws, wsb, stream, 0);
}
int sht_analyze(sht_plan_t plan, const double* grid, double* coeff, int F, void* ws, size_t wsb,
                void* stream) {
  return traced_transform("sht_analyze", plan, plan ? plan->precision : SHT_FP64, grid, coeff, F, ws, wsb, stream, 1);
}
int sht_synth_adjoint(sht_plan_t plan, const double* grid_cot, double* coeff_cot, int F, void* ws,
                      size_t wsb, void* stream) {
  return traced_transform("sht_synth_adjoint", plan, plan ? plan->precision : SHT_FP64, grid_cot, coeff_cot, F, ws,
                          wsb, stream, 2);
}
int sht_synth_ex(sht_plan_t plan, int prec, const double* coeff, double* grid, int F, void* ws,
                 size_t wsb, void* stream) {
  return traced_transform("sht_synth_ex", plan, prec, coeff, grid, F, ws, wsb, stream, 0);
}
int sht_analyze_ex(sht_plan_t plan, int prec, const double* grid, double* coeff, int F, void* ws,
                   size_t wsb, void* stream) {
  return traced_transform("sht_analyze_ex", plan, prec, grid, coeff, F, ws, wsb, stream, 1);
}
int sht_synth_adjoint_ex(sht_plan_t plan, int prec, const double* grid_cot, double* coeff_cot, int F,
                         void* ws, size_t wsb, void* stream) {
  return traced_transform("sht_synth_adjoint_ex", plan, prec, grid_cot, coeff_cot, F, ws, wsb, stream, 2);
}

int sht_plan_stats(sht_plan_t plan, sht_stats* out) {
  if (!plan || !out) return SHT_EINVAL;
  *out = plan->stats;
  return SHT_OK;
}

int sht_profile_enable(sht_plan_t plan, int enable) {
  if (!plan) return SHT_EINVAL;
  DeviceScope ds(plan->device);
  if (!enable) (void)plan->prof.flush();
  plan->prof.on = enable != 0;
  return SHT_OK;
}

int sht_profile_reset(sht_plan_t plan) {
  if (!plan) return SHT_EINVAL;
  DeviceScope ds(plan->device);
  plan->prof.clear();
  return SHT_OK;
}

int sht_profile_count(sht_plan_t plan) {
  if (!plan) return SHT_EINVAL;
  DeviceScope ds(plan->device);
  const int rc = plan->prof.flush();
  if (rc != SHT_OK) return rc;
  return static_cast<int>(plan->prof.recs.size());
}

int sht_profile_get(sht_plan_t plan, int i, const char** name, double* total_ms,
                    long long* launches, double* flops_per_launch, double* bytes_per_launch) {
  if (!plan || i < 0 || i >= static_cast<int>(plan->prof.recs.size())) return SHT_EINVAL;
  const ProfRecord& r = plan->prof.recs[i];
  if (name) *name = r.name.c_str();
  if (total_ms) *total_ms = r.ms;
  if (launches) *launches = r.launches;
  if (flops_per_launch) *flops_per_launch = r.flops;
  if (bytes_per_launch) *bytes_per_launch = r.bytes;
  return SHT_OK;
}

long long sht_num_coeffs(int l, int kind) {
  if (l < 1) return -1;
  return kind == SHT_REAL ? 2LL * l * l + l : 4LL * l * l;
}

long long sht_coeff_index(int l, int k, int m, int kind) {
  const int am = m < 0 ? -m : m;
  if (l < 1 || am > k || k > 2 * l - 1) return -1;
  const long long L2 = 2LL * l;
  if (kind == SHT_REAL) {
    if (m < 0) return -1;
    return static_cast<long long>(am) * L2 - static_cast<long long>(am) * (am - 1) / 2 + (k - am);
  }
  long long base = am == 0 ? 0 : L2 + 2LL * (am - 1) * L2 - static_cast<long long>(am - 1) * am;
  if (m < 0) base += L2 - am;
  return base + (k - am);
}

int sht_gl_nodes(int n, double* x, double* w) {
  if (n < 1 || !x || !w) return SHT_EINVAL;
  gauss_legendre(n, x, w);
  return SHT_OK;
}

int sht_plan_tree(sht_plan_t plan, int m, int p, int* levels, int* n_cols) {
  if (!plan || m < 0 || m >= 2 * plan->l || (p != 0 && p != 1)) return SHT_EINVAL;
  if (levels) *levels = plan->levels[2 * m + p];
  if (n_cols) *n_cols = plan->n_cols[2 * m + p];
  return SHT_OK;
}

int sht_plan_columns(sht_plan_t plan, int m, int p, double* q, int ldq) {
  if (!plan || plan->maps || !q || m < 0 || m >= 2 * plan->l || (p != 0 && p != 1) || ldq < plan->l)
    return SHT_EINVAL;
  DeviceScope ds(plan->device);
  if (!ds.ok()) return SHT_EHIP;
  const int l = plan->l, C = plan->C, n = plan->n_cols[2 * m + p];
  if (n == 0) return SHT_OK;
  const int leaves = (n + C - 1) / C;
  ColumnBatch cb;
  cb.npairs = 1;
  cb.l = l;
  cb.C = C;
  std::vector<double> sw(l);
  for (int i = 0; i < l; ++i) sw[i] = std::sqrt(2.0 * plan->wp[i]);
  void *dm = nullptr, *dp = nullptr, *dn = nullptr, *dprev = nullptr, *dcur = nullptr,
       *dexp = nullptr, *dout = nullptr, *dx = nullptr, *dsw = nullptr;
  int rc = SHT_OK;
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess && rc == SHT_OK) rc = SHT_EHIP;
    return rc == SHT_OK;
  };
  if (ok(dev_alloc(&dm, 4)) && ok(dev_alloc(&dp, 4)) && ok(dev_alloc(&dn, 4)) &&
      ok(dev_alloc(&dprev, 16 * l)) && ok(dev_alloc(&dcur, 16 * l)) && ok(dev_alloc(&dexp, 4 * l)) &&
      ok(dev_alloc(&dout, 8 * static_cast<size_t>(C) * l)) && ok(dev_alloc(&dx, 8 * l)) &&
      ok(dev_alloc(&dsw, 8 * l)) && ok(hipMemcpy(dm, &m, 4, hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dp, &p, 4, hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dn, &n, 4, hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dx, plan->xp.data(), 8 * l, hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dsw, sw.data(), 8 * l, hipMemcpyHostToDevice))) {
    cb.d_m = static_cast<int*>(dm);
    cb.d_p = static_cast<int*>(dp);
    cb.d_ncols = static_cast<int*>(dn);
    cb.d_prev = static_cast<double*>(dprev);
    cb.d_cur = static_cast<double*>(dcur);
    cb.d_exp = static_cast<int*>(dexp);
    cb.d_out = static_cast<double*>(dout);
    cb.d_x = static_cast<const double*>(dx);
    cb.d_sw = static_cast<const double*>(dsw);
    std::vector<double> chunk(static_cast<size_t>(C) * l);
    if (ok(legendre_seed(cb, nullptr))) {
      for (int c = 0; c < leaves && rc == SHT_OK; ++c) {
        if (!ok(legendre_chunk(cb, c, nullptr))) break;
        if (!ok(hipMemcpy(chunk.data(), dout, 8 * chunk.size(), hipMemcpyDeviceToHost))) break;
        const int width = std::min(C, n - c * C);
        for (int jj = 0; jj < width; ++jj)
          std::memcpy(q + static_cast<size_t>(c * C + jj) * ldq, chunk.data() + static_cast<size_t>(jj) * l,
                      8 * l);
      }
    }
  }
  for (void* ptr : {dm, dp, dn, dprev, dcur, dexp, dout, dx, dsw})
    if (ptr) (void)hipFree(ptr);
  return rc;
}

int sht_dense_q(sht_plan_t plan, int mp0, int count, double* q, long long stride, void* stream) {
  if (!plan || plan->maps || !q || count < 1 || mp0 < 0 || mp0 + count > 4 * plan->l ||
      stride < static_cast<long long>(plan->l) * plan->l)
    return SHT_EINVAL;
  DeviceScope ds(plan->device);
  if (!ds.ok()) return SHT_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int l = plan->l, C = plan->C;
  std::vector<int> hm(count), hp(count), hn(count);
  int nmax = 0;
  for (int i = 0; i < count; ++i) {
    hm[i] = (mp0 + i) / 2;
    hp[i] = (mp0 + i) % 2;
    hn[i] = plan->n_cols[mp0 + i];
    nmax = std::max(nmax, hn[i]);
  }
  if (nmax == 0) return SHT_OK;
  std::vector<double> sw(l);
  for (int i = 0; i < l; ++i) sw[i] = std::sqrt(2.0 * plan->wp[i]);
  void *dm = nullptr, *dp = nullptr, *dn = nullptr, *dprev = nullptr, *dcur = nullptr,
       *dexp = nullptr, *dout = nullptr, *dx = nullptr, *dsw = nullptr;
  int rc = SHT_OK;
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess && rc == SHT_OK) rc = SHT_EHIP;
    return rc == SHT_OK;
  };
  const size_t nc = static_cast<size_t>(count);
  if (ok(dev_alloc(&dm, 4 * nc)) && ok(dev_alloc(&dp, 4 * nc)) && ok(dev_alloc(&dn, 4 * nc)) &&
      ok(dev_alloc(&dprev, 16 * nc * l)) && ok(dev_alloc(&dcur, 16 * nc * l)) &&
      ok(dev_alloc(&dexp, 4 * nc * l)) && ok(dev_alloc(&dout, 8 * nc * C * l)) &&
      ok(dev_alloc(&dx, 8 * static_cast<size_t>(l))) && ok(dev_alloc(&dsw, 8 * static_cast<size_t>(l))) &&
      ok(hipMemcpy(dm, hm.data(), 4 * nc, hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dp, hp.data(), 4 * nc, hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dn, hn.data(), 4 * nc, hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dx, plan->xp.data(), 8 * static_cast<size_t>(l), hipMemcpyHostToDevice)) &&
      ok(hipMemcpy(dsw, sw.data(), 8 * static_cast<size_t>(l), hipMemcpyHostToDevice))) {
    ColumnBatch cb;
    cb.npairs = count;
    cb.l = l;
    cb.C = C;
    cb.d_m = static_cast<int*>(dm);
    cb.d_p = static_cast<int*>(dp);
    cb.d_ncols = static_cast<int*>(dn);
    cb.d_prev = static_cast<double*>(dprev);
    cb.d_cur = static_cast<double*>(dcur);
    cb.d_exp = static_cast<int*>(dexp);
    cb.d_out = static_cast<double*>(dout);
    cb.d_x = static_cast<const double*>(dx);
    cb.d_sw = static_cast<const double*>(dsw);
    if (ok(legendre_seed(cb, s))) {
      const int leaves = (nmax + C - 1) / C;
      for (int c = 0; c < leaves && rc == SHT_OK; ++c) {
        if (!ok(legendre_chunk(cb, c, s))) break;
        for (int i = 0; i < count && rc == SHT_OK; ++i) {
          const int width = std::min(C, hn[i] - c * C);
          if (width <= 0) continue;
          ok(hipMemcpyAsync(q + i * stride + static_cast<long long>(c) * C * l,
                            static_cast<double*>(dout) + static_cast<size_t>(i) * C * l,
                            8 * static_cast<size_t>(width) * l, hipMemcpyDeviceToDevice, s));
        }
      }
    }
    if (rc == SHT_OK) ok(hipStreamSynchronize(s));
  }
  for (void* ptr : {dm, dp, dn, dprev, dcur, dexp, dout, dx, dsw})
    if (ptr) (void)hipFree(ptr);
  return rc;
}

// ---- host-only builder -------------------------------------------------------------------

int sht_bf_build(const double* a, int rows, int cols, int lda, int leaf_width, int levels,
                 double eps, sht_bf_t* out) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (rows < 1 || cols < 0 || lda < rows || leaf_width < 1 || !(eps > 0.0) || (!a && cols > 0))
    return SHT_EINVAL;
  int L = levels < 0 ? butterfly_depth(cols, leaf_width) : levels;
  if (L > 24 || (1LL << L) * leaf_width < cols || (1LL << L) > rows) return SHT_EINVAL;
  sht_bf_s* bf = new (std::nothrow) sht_bf_s();
  if (!bf) return SHT_ENOMEM;
  try {
    bf->tree.init(rows, cols, leaf_width, L, eps);
    for (int c = 0; c < (1 << L); ++c) {
      const double* chunk = a ? a + static_cast<size_t>(c) * leaf_width * lda : nullptr;
      if (bf->tree.leaf_width(c) == 0) chunk = a;
      bf->tree.add_leaf(c, chunk, lda);
    }
  } catch (const std::bad_alloc&) {
    delete bf;
    return SHT_ENOMEM;
  } catch (...) {
    delete bf;
    return SHT_EINTERNAL;
  }
  *out = bf;
  return SHT_OK;
}

void sht_bf_destroy(sht_bf_t bf) { delete bf; }

int sht_plan_cache_check(const char* cache_dir, int l, double eps, int leaf_width, long long* valid_pairs) {
  if (valid_pairs) *valid_pairs = 0;
  if (!cache_dir || l < 1 || leaf_width < 1 || !(eps > 0.0 && eps < 1.0)) return SHT_EINVAL;
  CacheScan scan;
  const int rc = cache_scan(cache_dir, l, eps, leaf_width, 4 * l, nullptr, nullptr, scan);
  if (valid_pairs) *valid_pairs = scan.valid_pairs;
  return rc;
}

int sht_plan_cache_read(const char* cache_dir, int l, double eps, int leaf_width, int mp, sht_bf_t* out) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (!cache_dir || l < 1 || leaf_width < 1 || !(eps > 0.0 && eps < 1.0) || mp < 0 || mp >= 4 * l)
    return SHT_EINVAL;
  try {
    std::vector<PairShape> shapes(4 * l);
    for (int q = 0; q < 4 * l; ++q) shapes[q] = pair_shape(l, leaf_width, q);
    std::vector<BfTree> trees(4 * l);
    CacheScan scan;
    const int rc = cache_scan(cache_dir, l, eps, leaf_width, 4 * l, &shapes, &trees, scan);
    if (scan.valid_pairs <= mp) return rc == SHT_ECORRUPT ? SHT_ECORRUPT : SHT_EINVAL;
    sht_bf_s* bf = new sht_bf_s();
    bf->tree = std::move(trees[mp]);
    *out = bf;
    return SHT_OK;
  } catch (const std::bad_alloc&) {
    return SHT_ENOMEM;
  }
}

int sht_plan_cache_append(const char* cache_dir, int l, double eps, int leaf_width, int mp, sht_bf_t bf) {
  if (!cache_dir || !bf || l < 1 || leaf_width < 1 || !(eps > 0.0 && eps < 1.0) || mp < 0 || mp >= 4 * l)
    return SHT_EINVAL;
  const PairShape sh = pair_shape(l, leaf_width, mp);
  const BfTree& t = bf->tree;
  if (t.rows() != sh.rows || t.cols() != sh.cols || t.L() != sh.L || t.C() != leaf_width || !t.complete())
    return SHT_EINVAL;
  CacheScan scan;
  const int rc = cache_scan(cache_dir, l, eps, leaf_width, 4 * l, nullptr, nullptr, scan);
  if (rc == SHT_ECORRUPT) return SHT_ECORRUPT;
  if (mp != scan.valid_pairs) return SHT_EINVAL;
  try {
    CacheWriter w;
    int e = w.open(cache_dir, l, eps, leaf_width, 4 * l, scan.valid_bytes);
    if (e == SHT_OK) e = w.append(mp, t);
    if (e == SHT_OK) e = w.flush();
    return e;
  } catch (const std::bad_alloc&) {
    return SHT_ENOMEM;
  }
}

int sht_bf_info(sht_bf_t bf, int* levels, int* k_max, double* k_avg, double* k_sd,
                long long* factor_entries, long long* m_max_words) {
  if (!bf) return SHT_EINVAL;
  const BfTree& t = bf->tree;
  if (levels) *levels = t.L();
  if (k_max) *k_max = t.k_max;
  const double avg = t.n_ids ? t.sum_k / t.n_ids : 0.0;
  if (k_avg) *k_avg = avg;
  if (k_sd) *k_sd = t.n_ids ? std::sqrt(std::max(0.0, t.sum_k2 / t.n_ids - avg * avg)) : 0.0;
  if (factor_entries) *factor_entries = t.factor_entries;
  if (m_max_words) *m_max_words = t.m_max_words;
  return SHT_OK;
}

int sht_bf_block(sht_bf_t bf, int t, int r, int c, int* k, int* K, const int** skel,
                 const int** red, const double** T) {
  if (!bf) return SHT_EINVAL;
  const BfTree& tr = bf->tree;
  if (t < 0 || t > tr.L() || r < 0 || r >= tr.nrow(t) || c < 0 || c >= tr.ncol(t)) return SHT_EINVAL;
  const BfBlock& b = tr.block(t, r, c);
  if (k) *k = b.k;
  if (K) *K = b.K;
  if (skel) *skel = b.skel.data();
  if (red) *red = b.red.data();
  if (T) *T = b.T.data();
  return SHT_OK;
}

int sht_bf_final(sht_bf_t bf, int r, int* row0, int* h, int* k, const double** S, const int** cols) {
  if (!bf) return SHT_EINVAL;
  const BfTree& tr = bf->tree;
  if (r < 0 || r >= (1 << tr.L())) return SHT_EINVAL;
  const BfFinal& f = tr.final_block(r);
  if (row0) *row0 = f.row0;
  if (h) *h = f.h;
  if (k) *k = f.k;
  if (S) *S = f.S.data();
  if (cols) *cols = f.cols.data();
  return SHT_OK;
}

const char* sht_strerror(int status) {
  switch (status) {
    case SHT_OK: return "success";
    case SHT_EINVAL: return "invalid argument";
    case SHT_ENOMEM: return "out of memory";
    case SHT_EHIP: return "HIP runtime error";
    case SHT_EUNSUPPORTED: return "unsupported configuration";
    case SHT_EINTERNAL: return "internal error";
    case SHT_ENOTREADY: return "plan not prepared for this precision (sht_plan_prepare)";
    case SHT_ECORRUPT: return "plan cache file corrupt";
    default: return "unknown status";
  }
}

const char* sht_version(void) { return "0.1.0"; }

}  // extern "C"
