// Internal types shared by the host plan and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "sht.h"

namespace sht {

// Int8-slice form: where one stored matrix M (rows x cols) lives in the int8 pools, in the
// orientation each direction contracts with: 0 = M itself (synthesis), 1 = M^T (transposed
// apply).  Both are tile-packed signed 8-bit digits (16 rows x 64 contraction indices x the
// digits per 5 KiB block) with one int16 exponent per (padded) row.
struct I8Off {
  int64_t dig[2];  // byte offsets of the digit tiles of M and of M^T
  int64_t ex[2];   // offsets (int16 units) of the row exponents of M and of M^T
};

// One butterfly interpolation task: a leaf ID (one output) or a merged pair of
// row-split IDs that share their input (two outputs, top and bottom; Section
// 2.2 equations (top), (bottom)).  Rows are indices of R-wide rows in the
// workspace buffers.  Synthesis reads `in_row` and writes `out_row[]`; the
// transposed apply reads `out_row[]` and writes `in_row`.
struct LevelTask {
  int32_t in_row;     // first row of the input (concatenated children, or leaf columns)
  int32_t K;          // input length
  int32_t out_row[2]; // first row of each output block
  int32_t k[2];       // rank of each output block; k[1] = -1 for a leaf
  int32_t idx[2];     // offset of [skel (k) | red (K-k)] in the index pool
  int32_t mp;         // pair index 2m + p if the input rows are coefficients (leaf tasks, and
                      // level-1 tasks over folded identity leaves), else -1
  int64_t fac[2];     // offset of T (k x (K-k), column-major) in the factor pool
  I8Off i8[2];        // the same T in the int8-slice pools
};

// Position of Re/Im part `c` of beta_k^{+-m} (s = 0: +m, s = 1: -m) of field f in the
// canonical coefficient layout (orders ascending, +m block then -m block, degrees
// contiguous; real fields store m >= 0 only).
__host__ __device__ inline long long coeff_pos(int l, int kind, long long ncoef, int f, int m, int s,
                                               int k, int c) {
  const long long L2 = 2LL * l;
  long long base;
  if (kind == SHT_REAL) {
    base = static_cast<long long>(m) * L2 - static_cast<long long>(m) * (m - 1) / 2;
  } else {
    base = m == 0 ? 0 : L2 + 2LL * (m - 1) * L2 - static_cast<long long>(m - 1) * m;
    if (s) base += L2 - m;
  }
  return (static_cast<long long>(f) * ncoef + base + (k - m)) * 2 + c;
}

// Row of Y (the Legendre output and FFT input, R doubles wide) that holds order m on ring
// `ring`.  Ring-major: the 2l orders of one ring, which one FFT row reads, form one
// contiguous block of 2l rows, so an FFT work-group's gather stays within a few pages.
__host__ __device__ inline long long y_row(int l, int m, int ring) {
  return static_cast<long long>(ring) * (2LL * l) + m;
}

// Final skeleton product for one order m and one row node r at level L, both
// parities at once, followed by the parity unfold g(+-x) = E +- O and the row
// scaling D^{-1} (synthesis) or its transpose (analysis).
struct FinalTask {
  int32_t m;
  int32_t row0, h;    // positive-node rows [row0, row0 + h)
  int32_t k[2];       // ranks, parity 0 / 1
  int32_t in_row[2];  // V rows of the level-L blocks, parity 0 / 1
  int32_t vbuf;       // which V buffer holds them (L % 2)
  int32_t pad;
  int64_t fac[2];     // S (h x k, column-major) offsets
  I8Off i8[2];        // the same S in the int8-slice pools
};

// Final skeleton product of one per-order map (Section 5: the n x n matrix A^{(m,p)} of
// (transform) / (transform2) on its own nodes) and one row node r at level L: y = S w on
// rows [out_row, out_row + h) of the output, no parity unfold and no row scaling (the
// square roots of the weights are inside A).
struct OrderFinal {
  int32_t in_row;     // V rows of the level-L block
  int32_t out_row;    // first output row (pair base + row0)
  int32_t h, k;       // rows, rank
  int32_t vbuf;       // which V buffer holds the block (L % 2)
  int32_t pad;
  int64_t fac;        // S (h x k, column-major) offset; the transposed pool holds S^T there
};

// Layout descriptor of one (m, p) pair in the internal coefficient buffer.
struct PairDesc {
  int32_t m, p, n;    // order, parity, number of columns n_p
  int32_t in_base;    // first XIN row
};

// One stored factor matrix (T of an ID or S of a final skeleton), column-major.
struct FactorBlock {
  int64_t off;
  int32_t rows, cols;
};

// A stored matrix and its place in the int8-slice pools (input of the digit preparation).
struct I8Block {
  int64_t off;        // FP64 offset in the factor pool (column-major rows x cols)
  int32_t rows, cols;
  I8Off o;
};

// Int8-slice digits per entry and the highest product level kept (digit pairs s + u <= kI8Top
// of the kI8Dig x kI8Dig products; s = 0 is the most significant digit).
constexpr int kI8Dig = 6;
constexpr int kI8Top = 5;
// Bytes of the digit tiles of an A operand with `rows` rows and `kd` contraction indices.
inline long long i8_tile_bytes(long long rows, long long kd) {
  return ((rows + 15) / 16) * ((kd + 63) / 64) * kI8Dig * 1024LL;
}
inline long long i8_exp_count(long long rows) { return ((rows + 15) / 16) * 16; }

struct DeviceFactors {
  double* fac = nullptr;       // T and S entries (FP64), column-major, read by synthesis
  double* fac_t = nullptr;     // the same matrices transposed (same offsets), read by analysis
  float2* fac_hl = nullptr;    // split copies (first use of a split/FP32 transform): per entry
                               // the leading slice on its row's grid and the FP32 remainder
  float2* fac_t_hl = nullptr;  // the same for the transposed copies
  int8_t* dig = nullptr;       // int8-slice digit tiles, both orientations (sht_plan_prepare)
  int16_t* dex = nullptr;      // their row exponents
  I8Block* i8blocks = nullptr; // every stored matrix with its int8 offsets (for the preparation)
  FactorBlock* blocks = nullptr;  // every stored matrix (offset, rows, cols)
  uint16_t* idx = nullptr;     // skel/red index lists
  LevelTask* tasks = nullptr;  // all level tasks, step by step
  FinalTask* finals = nullptr;
  OrderFinal* ofinals = nullptr;  // per-order map plans: final skeletons, one per (pair, row node)
  PairDesc* pairs = nullptr;
  double* invD = nullptr;      // 1 / sqrt(2 w_i) on the positive nodes
  double* D = nullptr;         // sqrt(2 w_i)
  double* twiddle = nullptr;   // e^{2 pi i j / N}, j = 0..N-1 (interleaved)
};

// Optional per-stage timing: HIP events recorded around every kernel launch of a
// transform on the caller's stream, accumulated by stage name when read.
struct ProfRecord {
  std::string name;
  double ms = 0.0;
  long long launches = 0;
  double flops = 0.0;  // algorithmic flops per launch
  double bytes = 0.0;  // algorithmic HBM bytes per launch
};
struct ProfPending {
  int rec;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  std::vector<ProfRecord> recs;
  std::vector<ProfPending> pending;
  int find_or_add(const std::string& name, double flops, double bytes);
  int flush();  // waits for the recorded events and accumulates their times
  void clear();
};

// A contiguous run of tasks of one step launched together (one LDS size).
struct LaunchClass {
  long long off, cnt;  // task range relative to the step's first task
  int maxK, maxk;      // largest input length and output rank in the range
  int cls;
  int maxnr = 0;       // largest contraction length of the synthesis orientation (K - k;
                       // finals: largest rank) in the range
  // algorithmic work per R column: factor entries, vector rows read and written
  double fac = 0.0, rows_in = 0.0, rows_out = 0.0;
};

// Factor entries in the orientation a transform reads: FP64, and the split copies.
struct FacPtr {
  const double* d;   // FP64 entries
  const float2* hl;  // split: (leading slice on the row's grid, fp32 remainder) per entry
};

// Where a leaf task's vector rows live when they are read from / written to the caller's
// coefficients directly (the layout change fused into the leaf level): one contiguous
// [field][ncoef] array, or one base pointer per field (null entries: padding columns).
struct CoefIO {
  double* coeff;         // contiguous array, or null
  double* const* fptr;   // per-field base pointers, or null
  long long ncoef;
  int l, kind;
  __device__ bool on() const { return coeff != nullptr || fptr != nullptr; }
  __device__ double* at(int f, int m, int s, int k, int c) const {
    if (fptr) {
      double* b = fptr[f];
      return b ? b + coeff_pos(l, kind, 0, 0, m, s, k, c) : nullptr;
    }
    return coeff + coeff_pos(l, kind, ncoef, f, m, s, k, c);
  }
};

// Batched execution: one group = one plan and a set of fields (R columns, padded), with its
// own workspace; one item = one (task, column block) of one group.
struct BatchGroupDev {
  const LevelTask* tasks;
  const FinalTask* finals;
  FacPtr fp;                // orientation read by this direction
  const uint16_t* idx;
  const PairDesc* pairs;
  const double* rowscale;   // synthesis: 1/D; analysis: D; adjoint: 1/D
  double half;              // transposed final: 1/2 (analysis) or 1 (adjoint)
  double* v0;
  double* v1;
  double* y;
  CoefIO io;
  int R, l;
};
enum { kItemLevel = 0, kItemFinal = 1 };
struct BatchItem {
  int32_t group;
  int16_t kind;   // kItemLevel / kItemFinal
  int16_t step;   // level step t
  int32_t blk;    // column block
  int32_t pad;
  int64_t task;   // index into the plan's level tasks / finals
};
// Arguments of the persistent kernel: phases run in order with a grid-wide barrier between
// them; the items of (phase, queue) are items[qoff[phase * nq + q] .. qoff[phase * nq + q + 1]);
// sync holds one head counter per (phase, queue) then one barrier counter per phase, all zero
// at launch; status is set to 1 if a barrier wait exceeds spin_limit polls.
struct BatchLaunch {
  const BatchGroupDev* groups;
  const BatchItem* items;
  const int* qoff;
  int nphase, nq;
  unsigned* sync;
  int* status;
  long long spin_limit;
};

}  // namespace sht

struct sht_plan_s {
  int l = 0;
  int C = 64;
  int Lmax = 0;
  int device = 0;
  int precision = SHT_FP64;
  int kind = SHT_COMPLEX;
  bool maps = false;  // a plan of the per-order maps of Section 5 (sht_order_plan), not of the SHT
  double eps = 0.0;
  std::vector<double> xp, wp;           // positive nodes ascending and their weights
  std::vector<int> n_cols, levels;      // per pair mp = 2m + p
  std::vector<int> in_base, v_base, v_rows;
  long long rows_in = 0, rows_v = 0, rows_y = 0;
  long long n_fac = 0, n_fac_split = 0, n_idx = 0, n_blocks = 0;
  long long n_dig = 0, n_dex = 0;       // int8-slice pool sizes (bytes, int16 exponents)
  std::vector<long long> step_off, step_cnt;  // level tasks per step (t = 0..Lmax)
  std::vector<int> step_maxK, step_maxk;      // largest input / output length per step
  std::vector<std::vector<sht::LaunchClass>> step_classes;
  std::vector<sht::LaunchClass> final_classes;  // maxK holds the largest row count h
  int final_maxk = 0, final_maxh = 0;
  // algorithmic work per step: factor entries, input rows, output rows (per R column)
  std::vector<double> step_fac, step_rows_in, step_rows_out;
  double final_fac = 0, final_rows_v = 0, final_rows_y = 0;
  sht::Profiler prof;
  long long n_final = 0;
  long long n_ofinal = 0;        // per-order map plans: OrderFinal count, largest rank and rows
  int ofinal_maxk = 0, ofinal_maxh = 0;
  long long n_pairs = 0;
  long long n_folded = 0;  // orders whose leaf step is folded into level 1
  sht::DeviceFactors d;
  std::mutex split_mu;  // serialises the one-time derivation of the split factor copies
  sht_stats stats{};
};

namespace sht {

// Kernel launchers (apply.hip, fft.hip, legendre_cols.hip).
hipError_t launch_coeff_to_xin(const sht_plan_s* P, const double* coeff, double* xin, int F,
                               int R, hipStream_t s);
hipError_t launch_xin_to_coeff(const sht_plan_s* P, const double* xin, double* coeff, int F,
                               int R, hipStream_t s);
// cls >= 0 (matrix-core path only): launch only that size class of the step / of the finals.
// Tasks whose input rows are coefficients (LevelTask::mp >= 0) read / write them through
// `coeff` (matrix-core path: the caller's layout) or `xin` (vector path: internal rows).
hipError_t launch_level(const sht_plan_s* P, int step, bool transpose, const double* in,
                        double* out, int R, int precision, hipStream_t s, double* coeff = nullptr,
                        int cls = -1, double* xin = nullptr);
hipError_t launch_final(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                        double* v0w, double* v1w, double* y, const double* yin, int R,
                        int precision, bool adjoint, hipStream_t s, int cls = -1);
// Per-order map plans (FP64): y rows = S w from V (synthesis direction), or V = S^T y rows.
hipError_t launch_order_final(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                              double* v0w, double* v1w, double* y, const double* yin, int R, hipStream_t s);
// fptr (may be null): one grid base pointer per field instead of a contiguous array.
hipError_t launch_fft_synth(const sht_plan_s* P, const double* y, double* grid, int F, int R,
                            hipStream_t s, double* const* fptr = nullptr);
hipError_t launch_fft_analyze(const sht_plan_s* P, const double* grid, double* y, int F, int R,
                              double scale, double real_pos, hipStream_t s,
                              double* const* fptr = nullptr);
// Synthesis (api.cpp) into the caller's workspace; allow_prof = false: no per-stage events.
int run_synth(sht_plan_s* P, int precision, const double* coeff, double* grid, int F, void* ws,
              size_t wsb, void* stream, bool allow_prof);
size_t synth_workspace_bytes(const sht_plan_s* P, int F);
hipError_t fft_prepare(int l);  // kernel attributes for 4l-point rows (before graph capture)
hipError_t split_factors(sht_plan_s* P, hipStream_t s);
// split_factors under the plan's lock: calls from several host threads derive the copies once.
hipError_t ensure_split_factors(sht_plan_s* P, hipStream_t s);
bool mfma_ok(int R);
// coeff (leaf step only, may be null): read the leaf input from (synthesis) or write the
// leaf output to (transposed) the caller's coefficient array instead of the row buffer.
hipError_t launch_level_mfma(const sht_plan_s* P, int step, bool transpose, const double* in,
                             double* out, int R, int precision, hipStream_t s, double* coeff,
                             int cls = -1);
hipError_t launch_final_mfma(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                             double* v0w, double* v1w, double* y, const double* yin, int R,
                             int precision, bool adjoint, hipStream_t s, int cls = -1);
// Int8-slice form (apply_i8.hip): digit pools of the plan (i8_prepare, synchronises s) and
// the level / final launches of one step (cls >= 0: that size class only).
hipError_t i8_prepare(sht_plan_s* P, hipStream_t s);
hipError_t launch_level_i8(const sht_plan_s* P, int step, bool transpose, const double* in, double* out, int R,
                           hipStream_t s, double* coeff, int cls);
hipError_t launch_final_i8(const sht_plan_s* P, bool transpose, const double* v0, const double* v1, double* v0w,
                           double* v1w, double* y, const double* yin, int R, bool adjoint, hipStream_t s, int cls);
hipError_t transpose_factors(const double* fac, double* fac_t, const FactorBlock* blocks,
                             long long nblocks, hipStream_t s);
// Persistent batched kernel (column tile nt = 16 or 32): sets the LDS attribute and returns
// how many work-groups of it fit on one compute unit with `lds` bytes of dynamic LDS.
hipError_t batch_kernel_prepare(int nt, int precision, bool transpose, size_t lds, int* wg_per_cu);
hipError_t launch_batch_kernel(int nt, int precision, bool transpose, const BatchLaunch& bl,
                               unsigned grid, size_t lds, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, long long n, hipStream_t s);
size_t final_trans_lds_bytes();  // dynamic LDS of one transposed-final item

// Legendre column generator (legendre_cols.hip): recurrence state for a batch of pairs.
struct ColumnBatch {
  int npairs = 0, l = 0, C = 0;
  int* d_m = nullptr;
  int* d_p = nullptr;
  int* d_ncols = nullptr;
  double* d_prev = nullptr;    // npairs x l double-double values (2 doubles each)
  double* d_cur = nullptr;
  int* d_exp = nullptr;
  double* d_out = nullptr;     // npairs x C x l
  const double* d_x = nullptr; // positive nodes (l)
  const double* d_sw = nullptr;// sqrt(2 w)
};
hipError_t legendre_seed(ColumnBatch& b, hipStream_t s);
hipError_t legendre_chunk(ColumnBatch& b, int chunk, hipStream_t s);

void gauss_legendre(int n, double* x, double* w);

// Device-side IDs (id_device.hip).  One block: the h x K submatrix of a pair's Q on rows
// [row0, row0 + h) and the K global columns listed at gcols.
struct IdBlockDesc {
  int64_t q;      // offset of the pair's Q (column-major, leading dimension l) in the Q pool
  int64_t gcols;  // offset of the K column indices (also of the K output column order)
  int64_t work;   // offset of the block's h x K scratch
  int64_t tslot;  // offset of its T slot (K * K / 4 + 1 doubles)
  int32_t row0, h, K, pad;
};
// Appends the butterflies of pairs [first, end) to the plan cache (SHT_OK or a status).
using CacheAppend = std::function<int(int first, int end)>;
// Builds trees[first_pair ..] (pair mp = 2m + p of plan P, already sized) with every ID on
// the device, batch by batch; append (may be empty) runs after each batch.
class BfTree;
int build_trees_on_device(sht_plan_s* P, std::vector<BfTree>& trees, int first_pair, CacheAppend append,
                          double& t_cols, double& t_comp);

// ------------------------------------------------------------ allocation and call tracing
// Every device and pinned-host allocation of the library goes through dev_alloc /
// pinned_alloc.  Error-path tests: while an AllocFaultScope is alive (the entry points that
// build plans, factor copies and batches open one), SHT_TEST_FAIL_ALLOC_AFTER = n in the
// environment lets the first n allocations through and fails every later one with
// hipErrorOutOfMemory without touching the device.  Unset or negative: no failures.  Meant
// for one thread at a time.
hipError_t dev_alloc(void** p, size_t bytes);
hipError_t pinned_alloc(void** p, size_t bytes);
template <class T>
hipError_t dev_alloc(T** p, size_t bytes) {
  return dev_alloc(reinterpret_cast<void**>(p), bytes);
}
template <class T>
hipError_t pinned_alloc(T** p, size_t bytes) {
  return pinned_alloc(reinterpret_cast<void**>(p), bytes);
}
struct AllocFaultScope {
  AllocFaultScope();
  ~AllocFaultScope();
  AllocFaultScope(const AllocFaultScope&) = delete;
  AllocFaultScope& operator=(const AllocFaultScope&) = delete;
};

// Call tracing: SHT_TRACE = 1 (read on every call) writes one line per traced entry point to
// stderr (name, arguments, status, host time); SHT_TRACE = 2 also records events around a
// stream call, waits for the second and adds the device time.
class TraceCall {
 public:
  TraceCall(const char* name, int device, void* stream);
  ~TraceCall();
  TraceCall(const TraceCall&) = delete;
  TraceCall& operator=(const TraceCall&) = delete;
  bool on() const { return level_ > 0; }
  void args(const char* fmt, ...) __attribute__((format(printf, 2, 3)));
  int done(int rc);  // logs the call and returns rc

 private:
  const char* name_;
  int level_ = 0, device_ = -1;
  void* stream_ = nullptr;
  double t0_ = 0.0;
  hipEvent_t ev_[2] = {nullptr, nullptr};
  char args_[192] = {0};
};

}  // namespace sht
