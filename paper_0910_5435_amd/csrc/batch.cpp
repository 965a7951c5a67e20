// Batched execution of many transform requests: grouping, work lists, the persistent launch,
// graph capture and the autotuner (declared in include/sht.h).
//
// The butterfly of every order m, parity p, field and bandlimit is an independent chain of
// small interpolations (Section 3.2), so all of them can share the machine at once.  A
// batch merges the fields of requests that use the same plan into groups (R columns each),
// turns every (task, column block) of every group into a work item, and orders the items in
// phases: synthesis runs leaf, levels 1..L, final; the transposed directions run final,
// levels L..1, leaf.  Phase t of every group runs in the same phase of one persistent kernel,
// whose work-groups meet at a grid-wide barrier between phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sht_internal.h"

using namespace sht;

namespace {

constexpr int kMaxGroupCols = 512;
constexpr size_t kDefaultWsLimit = size_t(64) << 30;
constexpr long long kSpinLimit = 1LL << 21;  // barrier polls (~1-2 s) before giving up
constexpr size_t kMaxLds = 160 * 1024;

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }
int round_up(int v, int m) { return (v + m - 1) / m * m; }
int col_width(const sht_plan_s* P) { return P->kind == SHT_COMPLEX ? 4 : 2; }

struct Group {
  sht_plan_s* P = nullptr;
  std::vector<const void*> in;  // per field
  std::vector<void*> out;
  int F = 0;
  int Rmax = 0;  // columns padded to a multiple of 32 (the workspace stride bound)
  int set = 0;
  size_t ws_off = 0;
  double** d_in = nullptr;  // device pointer tables, Rmax / col_width entries
  double** d_out = nullptr;
};

size_t group_ws(const sht_plan_s* P, int R) {
  return 2 * a256(static_cast<size_t>(P->rows_v) * R * 8) + a256(static_cast<size_t>(P->rows_y) * R * 8);
}

struct SetDev {
  BatchGroupDev* groups = nullptr;
  BatchItem* items = nullptr;
  int* qoff = nullptr;
  long long nitems = 0;
  int nphase = 0;
  long long sync_off = 0;
  size_t lds = 0;
};

std::mutex g_tuned_mu;
std::map<std::string, sht_batch_config> g_tuned;

}  // namespace

struct sht_batch_s {
  int op = 0, precision = 0, device = 0, ncu = 0;
  std::vector<Group> groups;
  std::vector<std::vector<int>> sets;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int* d_status = nullptr;
  unsigned* d_sync = nullptr;
  long long n_sync = 0;
  std::vector<SetDev> sd;
  sht_batch_config cfg{};
  int grid = 0;
  long long items = 0, columns = 0;
  int max_phases = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string signature;
};

namespace {

bool trans_op(const sht_batch_s* B) { return B->op != SHT_BATCH_SYNTH; }

void free_lists(sht_batch_s* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  for (SetDev& s : B->sd) {
    (void)hipFree(s.groups);
    (void)hipFree(s.items);
    (void)hipFree(s.qoff);
  }
  B->sd.clear();
  (void)hipFree(B->d_sync);
  B->d_sync = nullptr;
  B->n_sync = 0;
}

void free_batch(sht_batch_s* B) {
  free_lists(B);
  for (Group& g : B->groups) {
    (void)hipFree(g.d_in);
    (void)hipFree(g.d_out);
  }
  (void)hipFree(B->ws);
  (void)hipFree(B->d_status);
}

// Largest input length of any level task and dynamic LDS of one item of a group.
size_t group_lds(const sht_plan_s* P, int nt, bool trans, int precision) {
  int maxK = 0;
  for (int v : P->step_maxK) maxK = std::max(maxK, v);
  (void)precision;  // transposed level items read their output vectors from global memory
  const size_t rows = static_cast<size_t>(maxK);
  size_t lds = (rows + 1) * (nt + 2) * 8 + 4 * static_cast<size_t>(maxK) + 16;  // + the zero row
  if (trans)
    lds = std::max(lds, final_trans_lds_bytes());
  else
    lds = std::max(lds, static_cast<size_t>(2 * P->final_maxk) * (nt + 2) * 8 + 16);
  return lds;
}

struct HostItem {
  BatchItem it;
  double cost;
};

// Items of one set for column tile nt: phase-major, then queue, each queue in decreasing
// cost; with nq = 8 all column blocks of a task go to the least-loaded queue.
int build_set(sht_batch_s* B, int si, int nt, int nq, SetDev& out, std::vector<BatchGroupDev>& gdev) {
  const bool trans = trans_op(B);
  const std::vector<int>& members = B->sets[si];
  int nphase = 0;
  for (int gi : members) nphase = std::max(nphase, B->groups[gi].P->Lmax + 2);
  std::vector<std::vector<HostItem>> per_phase(nphase);
  size_t lds = 0;
  gdev.clear();
  for (size_t local = 0; local < members.size(); ++local) {
    Group& g = B->groups[members[local]];
    const sht_plan_s* P = g.P;
    const int R = round_up(col_width(P) * g.F, nt);
    const int Rf = trans ? round_up(col_width(P) * g.F, 16) : R;
    if (Rf > R) return SHT_EINTERNAL;
    lds = std::max(lds, group_lds(P, nt, trans, B->precision));
    BatchGroupDev d{};
    d.tasks = P->d.tasks;
    d.finals = P->d.finals;
    d.fp = trans ? FacPtr{P->d.fac_t, P->d.fac_t_hl} : FacPtr{P->d.fac, P->d.fac_hl};
    d.idx = P->d.idx;
    d.pairs = P->d.pairs;
    d.rowscale = B->op == SHT_BATCH_ANALYZE ? P->d.D : P->d.invD;
    d.half = B->op == SHT_BATCH_ANALYZE ? 0.5 : 1.0;
    char* base = B->ws + g.ws_off;
    d.v0 = reinterpret_cast<double*>(base);
    d.v1 = reinterpret_cast<double*>(base + a256(static_cast<size_t>(P->rows_v) * g.Rmax * 8));
    d.y = reinterpret_cast<double*>(base + 2 * a256(static_cast<size_t>(P->rows_v) * g.Rmax * 8));
    const long long ncoef = P->kind == SHT_COMPLEX ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l;
    d.io = CoefIO{nullptr, trans ? g.d_out : g.d_in, ncoef, P->l, P->kind};
    d.R = R;
    d.l = P->l;
    gdev.push_back(d);
    const int L = P->Lmax;
    auto add_level = [&](int t, int ph) {
      for (const LaunchClass& lc : P->step_classes[t]) {
        const double cost = static_cast<double>(lc.maxK) * std::max(1, lc.maxk) * nt;
        for (long long i = 0; i < lc.cnt; ++i)
          for (int b = 0; b < R / nt; ++b) {
            HostItem h;
            h.it = BatchItem{static_cast<int32_t>(local), kItemLevel, static_cast<int16_t>(t), b, 0,
                             P->step_off[t] + lc.off + i};
            h.cost = cost;
            per_phase[ph].push_back(h);
          }
      }
    };
    auto add_final = [&](int ph) {
      const int ntf = trans ? 16 : nt;
      for (const LaunchClass& lc : P->final_classes) {
        const double cost = static_cast<double>(lc.maxK) * 2.0 * std::max(1, lc.maxk) * ntf;
        for (long long i = 0; i < lc.cnt; ++i)
          for (int b = 0; b < Rf / ntf; ++b) {
            HostItem h;
            h.it = BatchItem{static_cast<int32_t>(local), kItemFinal, 0, b, 0, lc.off + i};
            h.cost = cost;
            per_phase[ph].push_back(h);
          }
      }
    };
    if (!trans) {
      for (int t = 0; t <= L; ++t) add_level(t, t);
      add_final(L + 1);
    } else {
      add_final(0);
      for (int t = L; t >= 0; --t) add_level(t, L + 1 - t);
    }
  }
  if (lds > kMaxLds) return SHT_EINVAL;
  // queues
  std::vector<BatchItem> items;
  std::vector<int> qoff;
  qoff.push_back(0);
  for (int ph = 0; ph < nphase; ++ph) {
    std::vector<HostItem>& v = per_phase[ph];
    std::stable_sort(v.begin(), v.end(), [](const HostItem& a, const HostItem& b) { return a.cost > b.cost; });
    std::vector<std::vector<BatchItem>> q(nq);
    std::vector<double> load(nq, 0.0);
    size_t i = 0;
    while (i < v.size()) {  // the column blocks of one task are consecutive
      size_t j = i + 1;
      while (j < v.size() && v[j].it.group == v[i].it.group && v[j].it.kind == v[i].it.kind &&
             v[j].it.task == v[i].it.task)
        ++j;
      const int dst = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      for (size_t e = i; e < j; ++e) {
        q[dst].push_back(v[e].it);
        load[dst] += v[e].cost;
      }
      i = j;
    }
    for (int x = 0; x < nq; ++x) {
      items.insert(items.end(), q[x].begin(), q[x].end());
      qoff.push_back(static_cast<int>(items.size()));
    }
  }
  if (items.size() > static_cast<size_t>(1 << 30)) return SHT_EUNSUPPORTED;
  out.nphase = nphase;
  out.nitems = static_cast<long long>(items.size());
  out.lds = lds;
  if (dev_alloc(reinterpret_cast<void**>(&out.groups), gdev.size() * sizeof(BatchGroupDev)) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&out.items), std::max<size_t>(1, items.size()) * sizeof(BatchItem)) != hipSuccess ||
      dev_alloc(reinterpret_cast<void**>(&out.qoff), qoff.size() * sizeof(int)) != hipSuccess)
    return SHT_ENOMEM;
  if (hipMemcpy(out.groups, gdev.data(), gdev.size() * sizeof(BatchGroupDev), hipMemcpyHostToDevice) != hipSuccess ||
      (!items.empty() &&
       hipMemcpy(out.items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(out.qoff, qoff.data(), qoff.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return SHT_EHIP;
  return SHT_OK;
}

int configure(sht_batch_s* B, const sht_batch_config& c) {
  if (c.column_tile != 16 && c.column_tile != 32) return SHT_EINVAL;
  if (c.queues != 1 && c.queues != 8) return SHT_EINVAL;
  if (c.wg_per_cu < 1) return SHT_EINVAL;
  free_lists(B);
  const bool trans = trans_op(B);
  const int nt = c.column_tile, nq = c.queues;
  B->sd.resize(B->sets.size());
  std::vector<std::vector<BatchGroupDev>> gdevs(B->sets.size());
  size_t lds_max = 0;
  long long nsync = 0;
  B->items = 0;
  B->max_phases = 0;
  for (size_t si = 0; si < B->sets.size(); ++si) {
    const int rc = build_set(B, static_cast<int>(si), nt, nq, B->sd[si], gdevs[si]);
    if (rc != SHT_OK) {
      free_lists(B);
      return rc;
    }
    B->sd[si].sync_off = nsync;
    nsync += static_cast<long long>(B->sd[si].nphase) * (nq + 1);
    lds_max = std::max(lds_max, B->sd[si].lds);
    B->items += B->sd[si].nitems;
    B->max_phases = std::max(B->max_phases, B->sd[si].nphase);
  }
  int fit = 0;
  if (batch_kernel_prepare(nt, B->precision, trans, lds_max, &fit) != hipSuccess) {
    free_lists(B);
    return SHT_EHIP;
  }
  if (fit < c.wg_per_cu) {
    free_lists(B);
    return SHT_EINVAL;
  }
  for (Group& g : B->groups)
    if (fft_prepare(g.P->l) != hipSuccess) {
      free_lists(B);
      return SHT_EHIP;
    }
  B->n_sync = nsync;
  if (dev_alloc(reinterpret_cast<void**>(&B->d_sync), static_cast<size_t>(nsync + 1) * sizeof(unsigned)) != hipSuccess) {
    free_lists(B);
    return SHT_ENOMEM;
  }
  B->grid = B->ncu * c.wg_per_cu;
  // capture: reset counters, then per set the FFTs and the persistent kernel in order
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    free_lists(B);
    return SHT_EHIP;
  }
  int rc = SHT_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = SHT_EHIP;
  if (rc == SHT_OK && launch_fill_u32(B->d_sync, nsync, cs) != hipSuccess) rc = SHT_EHIP;
  if (rc == SHT_OK && launch_fill_u32(reinterpret_cast<unsigned*>(B->d_status), 1, cs) != hipSuccess)
    rc = SHT_EHIP;
  for (size_t si = 0; rc == SHT_OK && si < B->sets.size(); ++si) {
    const SetDev& s = B->sd[si];
    const std::vector<BatchGroupDev>& gd = gdevs[si];
    if (trans) {
      for (size_t k = 0; rc == SHT_OK && k < B->sets[si].size(); ++k) {
        const Group& g = B->groups[B->sets[si][k]];
        const bool adj = B->op == SHT_BATCH_ADJOINT;
        const double scale = adj ? 1.0 : 1.0 / (4.0 * g.P->l);
        if (launch_fft_analyze(g.P, nullptr, gd[k].y, g.F, gd[k].R, scale, adj ? 2.0 : 1.0, cs, g.d_in) !=
            hipSuccess)
          rc = SHT_EHIP;
      }
    }
    BatchLaunch bl{s.groups, s.items, s.qoff, s.nphase, nq, B->d_sync + s.sync_off, B->d_status, kSpinLimit};
    if (rc == SHT_OK && s.nitems > 0 &&
        launch_batch_kernel(nt, B->precision, trans, bl, static_cast<unsigned>(B->grid), lds_max, cs) != hipSuccess)
      rc = SHT_EHIP;
    if (!trans) {
      for (size_t k = 0; rc == SHT_OK && k < B->sets[si].size(); ++k) {
        const Group& g = B->groups[B->sets[si][k]];
        if (launch_fft_synth(g.P, gd[k].y, nullptr, g.F, gd[k].R, cs, g.d_out) != hipSuccess) rc = SHT_EHIP;
      }
    }
  }
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  if (rc == SHT_OK && ec != hipSuccess) rc = SHT_EHIP;
  (void)hipStreamDestroy(cs);
  if (rc == SHT_OK && hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = SHT_EHIP;
  B->graph = graph;
  if (rc != SHT_OK) {
    free_lists(B);
    return rc;
  }
  B->cfg = c;
  B->cfg.ms = 0.0;
  return SHT_OK;
}

}  // namespace

namespace {
int batch_create(const sht_request* reqs, int nreq, int op, int precision, size_t workspace_limit, void* stream,
                 sht_batch_t* out) {
  if (!out) return SHT_EINVAL;
  *out = nullptr;
  if (!reqs || nreq < 1) return SHT_EINVAL;
  if (op != SHT_BATCH_SYNTH && op != SHT_BATCH_ANALYZE && op != SHT_BATCH_ADJOINT) return SHT_EINVAL;
  if (precision == SHT_INT8) return SHT_EUNSUPPORTED;  // the persistent kernel has no int8 form
  if (precision != SHT_FP64 && precision != SHT_SPLIT32 && precision != SHT_FP32) return SHT_EINVAL;
  const size_t limit = workspace_limit ? workspace_limit : kDefaultWsLimit;
  int device = -1;
  for (int r = 0; r < nreq; ++r) {
    const sht_request& q = reqs[r];
    if (!q.plan || q.plan->maps || q.nfields < 1 || !q.input || !q.output) return SHT_EINVAL;
    if (reinterpret_cast<uintptr_t>(q.input) % 16 || reinterpret_cast<uintptr_t>(q.output) % 16)
      return SHT_EINVAL;
    if (device < 0) device = q.plan->device;
    if (q.plan->device != device) return SHT_EINVAL;
  }
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return SHT_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* B = new (std::nothrow) sht_batch_s;
  if (!B) return SHT_ENOMEM;
  B->op = op;
  B->precision = precision;
  B->device = device;
  int rc = SHT_OK;
  if (hipDeviceGetAttribute(&B->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || B->ncu < 1)
    rc = SHT_EHIP;
  // fields per plan, in request order, then chunks that fit the column and workspace limits
  std::vector<sht_plan_s*> plans;
  std::vector<std::vector<std::pair<const void*, void*>>> fields;
  for (int r = 0; rc == SHT_OK && r < nreq; ++r) {
    sht_plan_s* P = reqs[r].plan;
    size_t pi = std::find(plans.begin(), plans.end(), P) - plans.begin();
    if (pi == plans.size()) {
      plans.push_back(P);
      fields.emplace_back();
    }
    const bool cplx = P->kind == SHT_COMPLEX;
    const size_t in_field = trans_op(B) ? 2ull * P->l * 4ull * P->l * (cplx ? 16 : 8)
                                        : static_cast<size_t>(cplx ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l) * 16;
    const size_t out_field = trans_op(B) ? static_cast<size_t>(cplx ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l) * 16
                                         : 2ull * P->l * 4ull * P->l * (cplx ? 16 : 8);
    for (int f = 0; f < reqs[r].nfields; ++f)
      fields[pi].emplace_back(static_cast<const char*>(reqs[r].input) + f * in_field,
                              static_cast<char*>(reqs[r].output) + f * out_field);
  }
  for (size_t pi = 0; rc == SHT_OK && pi < plans.size(); ++pi) {
    sht_plan_s* P = plans[pi];
    const int cw = col_width(P);
    const size_t per_col = group_ws(P, 1);
    int max_cols = std::min<long long>(kMaxGroupCols, static_cast<long long>(limit / std::max<size_t>(per_col, 1)));
    max_cols = max_cols / 32 * 32;
    if (max_cols < 32) {
      rc = SHT_ENOMEM;
      break;
    }
    const int fmax = max_cols / cw;
    for (size_t f0 = 0; f0 < fields[pi].size(); f0 += fmax) {
      Group g;
      g.P = P;
      for (size_t f = f0; f < std::min(fields[pi].size(), f0 + fmax); ++f) {
        g.in.push_back(fields[pi][f].first);
        g.out.push_back(fields[pi][f].second);
      }
      g.F = static_cast<int>(g.in.size());
      g.Rmax = round_up(cw * g.F, 32);
      B->groups.push_back(std::move(g));
    }
    if (precision != SHT_FP64 && ensure_split_factors(P, s) != hipSuccess) rc = SHT_EHIP;
    if (precision == SHT_FP64 && !P->d.fac) rc = SHT_ENOTREADY;  // a split-only plan
  }
  // launch sets: largest workspaces first, first fit under the limit
  if (rc == SHT_OK) {
    std::vector<int> order(B->groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return group_ws(B->groups[a].P, B->groups[a].Rmax) > group_ws(B->groups[b].P, B->groups[b].Rmax);
    });
    std::vector<size_t> used;
    for (int gi : order) {
      const size_t w = group_ws(B->groups[gi].P, B->groups[gi].Rmax);
      size_t si = 0;
      while (si < used.size() && used[si] + w > limit) ++si;
      if (si == used.size()) {
        used.push_back(0);
        B->sets.emplace_back();
      }
      B->groups[gi].set = static_cast<int>(si);
      B->groups[gi].ws_off = used[si];
      used[si] += w;
      B->sets[si].push_back(gi);
    }
    for (size_t u : used) B->ws_bytes = std::max(B->ws_bytes, u);
    for (std::vector<int>& m : B->sets) std::sort(m.begin(), m.end());
  }
  if (rc == SHT_OK && (dev_alloc(reinterpret_cast<void**>(&B->ws), std::max<size_t>(B->ws_bytes, 256)) != hipSuccess ||
                       dev_alloc(reinterpret_cast<void**>(&B->d_status), sizeof(int)) != hipSuccess))
    rc = SHT_ENOMEM;
  // the Y rows of padding columns are never written by the transposed FFT: clear them once
  if (rc == SHT_OK && hipMemset(B->ws, 0, B->ws_bytes) != hipSuccess) rc = SHT_EHIP;
  if (rc == SHT_OK && hipMemset(B->d_status, 0, sizeof(int)) != hipSuccess) rc = SHT_EHIP;
  for (size_t gi = 0; rc == SHT_OK && gi < B->groups.size(); ++gi) {
    Group& g = B->groups[gi];
    const int n = g.Rmax / col_width(g.P);
    std::vector<double*> tin(n, nullptr), tout(n, nullptr);
    for (int f = 0; f < g.F; ++f) {
      tin[f] = const_cast<double*>(static_cast<const double*>(g.in[f]));
      tout[f] = static_cast<double*>(g.out[f]);
    }
    if (dev_alloc(reinterpret_cast<void**>(&g.d_in), n * sizeof(double*)) != hipSuccess ||
        dev_alloc(reinterpret_cast<void**>(&g.d_out), n * sizeof(double*)) != hipSuccess) {
      rc = SHT_ENOMEM;
      break;
    }
    if (hipMemcpy(g.d_in, tin.data(), n * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g.d_out, tout.data(), n * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess)
      rc = SHT_EHIP;
    B->columns += g.Rmax;
  }
  if (rc == SHT_OK) {
    B->signature = std::to_string(op) + "/" + std::to_string(precision);
    for (const Group& g : B->groups)
      B->signature += "|" + std::to_string(g.P->l) + "," + std::to_string(g.P->kind) + "," +
                      std::to_string(g.P->C) + "," + std::to_string(g.P->eps) + "," + std::to_string(g.Rmax);
    sht_batch_config c{16, 2, 8, 0.0};
    {
      std::lock_guard<std::mutex> lk(g_tuned_mu);
      auto it = g_tuned.find(B->signature);
      if (it != g_tuned.end()) c = it->second;
    }
    rc = configure(B, c);
    if (rc == SHT_EINVAL && c.wg_per_cu > 1) {  // fewer resident work-groups if LDS is short
      c.wg_per_cu = 1;
      rc = configure(B, c);
    }
  }
  if (rc == SHT_OK && hipDeviceSynchronize() != hipSuccess) rc = SHT_EHIP;
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rc != SHT_OK) {
    free_batch(B);
    delete B;
    return rc;
  }
  *out = B;
  return SHT_OK;
}

}  // namespace

extern "C" {

int sht_batch_create(const sht_request* reqs, int nreq, int op, int precision, size_t workspace_limit,
                     void* stream, sht_batch_t* out) {
  TraceCall tc("sht_batch_create", reqs && nreq > 0 && reqs[0].plan ? reqs[0].plan->device : -1, nullptr);
  if (tc.on()) tc.args("nreq=%d, op=%d, precision=%d", nreq, op, precision);
  AllocFaultScope faults;
  return tc.done(batch_create(reqs, nreq, op, precision, workspace_limit, stream, out));
}

int sht_batch_configure(sht_batch_t B, const sht_batch_config* cfg) {
  if (!B || !cfg) return SHT_EINVAL;
  sht_batch_config c = B->cfg;
  if (cfg->column_tile) c.column_tile = cfg->column_tile;
  if (cfg->wg_per_cu) c.wg_per_cu = cfg->wg_per_cu;
  if (cfg->queues) c.queues = cfg->queues;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(B->device) != hipSuccess) return SHT_EHIP;
  int rc = configure(B, c);
  if (rc != SHT_OK && configure(B, B->cfg.column_tile ? B->cfg : sht_batch_config{16, 1, 8, 0.0}) != SHT_OK)
    rc = SHT_EINTERNAL;  // the previous configuration could not be restored
  if (prev >= 0) (void)hipSetDevice(prev);
  return rc;
}

int sht_batch_run(sht_batch_t B, void* stream) {
  TraceCall tc("sht_batch_run", B ? B->device : -1, stream);
  if (!B || !B->exec) return tc.done(SHT_EINVAL);
  return tc.done(hipGraphLaunch(B->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? SHT_OK : SHT_EHIP);
}

int sht_batch_check(sht_batch_t B, void* stream) {
  if (!B) return SHT_EINVAL;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return SHT_EHIP;
  int st = 0;
  if (hipMemcpy(&st, B->d_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SHT_EHIP;
  return st ? SHT_EINTERNAL : SHT_OK;
}

int sht_batch_tune(sht_batch_t B, int reps, void* stream, sht_batch_config* best) {
  if (!B || reps < 1) return SHT_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SHT_EHIP;
  sht_batch_config win{0, 0, 0, 1e300};
  int rc = SHT_OK;
  for (int nt : {16, 32}) {
    for (int nq : {8, 1}) {
      for (int w = 1; w <= 4; ++w) {
        const sht_batch_config c{nt, w, nq, 0.0};
        if (configure(B, c) != SHT_OK) continue;  // does not fit: skip
        if (sht_batch_run(B, s) != SHT_OK || sht_batch_check(B, s) != SHT_OK) continue;
        float ms = 0.0f;
        if (hipEventRecord(e0, s) != hipSuccess) {
          rc = SHT_EHIP;
          break;
        }
        for (int r = 0; r < reps; ++r) (void)sht_batch_run(B, s);
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = SHT_EHIP;
          break;
        }
        if (sht_batch_check(B, s) != SHT_OK) continue;
        const double per = ms / reps;
        if (per < win.ms) win = sht_batch_config{nt, w, nq, per};
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SHT_OK) return rc;
  if (win.column_tile == 0) return SHT_EINTERNAL;
  rc = configure(B, win);
  if (rc != SHT_OK) return rc;
  B->cfg.ms = win.ms;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[B->signature] = win;
  }
  if (best) *best = win;
  return SHT_OK;
}

int sht_batch_get_info(sht_batch_t B, sht_batch_info* out) {
  if (!B || !out) return SHT_EINVAL;
  out->groups = static_cast<int>(B->groups.size());
  out->launches = static_cast<int>(B->sets.size());
  out->phases = B->max_phases;
  out->items = B->items;
  out->columns = B->columns;
  out->workspace_bytes = B->ws_bytes;
  out->config = B->cfg;
  out->grid = B->grid;
  return SHT_OK;
}

void sht_batch_destroy(sht_batch_t B) {
  if (!B) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(B->device);
  (void)hipDeviceSynchronize();
  free_batch(B);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete B;
}

}  // extern "C"
