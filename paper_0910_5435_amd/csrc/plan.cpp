// sht_plan: host FP64 precompute of the butterfly factors for every order m and
// parity p, and their upload in execution order.
//
//  1. Gauss-Legendre nodes (equation (thetas)); the l positive ones are the rows
//     of every Q^{(m,p)}, the diagonal sqrt(2 w) is kept outside the
//     compressed matrices (Remark omission).
//  2. Columns of Q^{(m,p)} come from the GPU recurrence kernel one leaf chunk at
//     a time, and each chunk is consumed at once by the depth-first butterfly
//     construction (Section 4), so no (m, p) ever holds its full matrix.
//  3. The resulting IDs are packed step by step (leaves, then each merge level,
//     then the final skeletons) so the apply kernels stream them in order; the
//     factor values go to the device as they are packed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "interp_decomp.h"
#include "plan_cache.h"
#include "sht_internal.h"

namespace sht {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

template <typename F>
void parallel_for(int n, int nthreads, F&& fn) {
  if (n <= 0) return;
  nthreads = std::max(1, std::min(nthreads, n));
  if (nthreads == 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  th.reserve(nthreads);
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&]() {
      for (int i = next++; i < n; i = next++) fn(i);
    });
  for (auto& x : th) x.join();
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// The factor pool goes to the device in pack order through two pinned staging buffers
// (one fills while the other is copied), so the host never holds the whole pool: at
// l = 1024 that pool is ~7.5 GB, whose first touch alone would cost seconds.  `dev` holds
// exactly `total` doubles; appending past it is refused rather than written.
class FactorStream {
 public:
  static constexpr size_t kCap = size_t(8) << 20;  // doubles per staging buffer (64 MB)
  FactorStream(double* dev, size_t total) : dev_(dev), total_(total) {
    for (int b = 0; b < 2; ++b) {
      if (err_ == hipSuccess)
        err_ = pinned_alloc(reinterpret_cast<void**>(&stage_[b]), kCap * sizeof(double));
      if (err_ == hipSuccess) err_ = hipEventCreateWithFlags(&ev_[b], hipEventDisableTiming);
    }
  }
  ~FactorStream() {
    (void)hipStreamSynchronize(nullptr);
    for (int b = 0; b < 2; ++b) {
      if (stage_[b]) (void)hipHostFree(stage_[b]);
      if (ev_[b]) (void)hipEventDestroy(ev_[b]);
    }
  }
  size_t size() const { return off_; }
  void append(const double* p, size_t n) {
    if (n == 0) return;
    if (off_ + n > total_) overrun_ = true;
    if (overrun_ || err_ != hipSuccess) {
      off_ += n;
      return;
    }
    while (n > 0 && err_ == hipSuccess) {
      const size_t take = std::min(n, kCap - fill_);
      std::memcpy(stage_[cur_] + fill_, p, take * sizeof(double));
      fill_ += take;
      p += take;
      n -= take;
      off_ += take;
      if (fill_ == kCap) flush();
    }
    off_ += n;  // what a copy error left unsent still counts
  }
  // SHT_OK once every appended value is on the device and the count is the one announced.
  int close() {
    flush();
    if (err_ == hipSuccess) err_ = hipStreamSynchronize(nullptr);
    if (err_ != hipSuccess) return err_ == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EHIP;
    return overrun_ || off_ != total_ ? SHT_EINTERNAL : SHT_OK;
  }

 private:
  void flush() {
    if (fill_ == 0) return;
    if (err_ == hipSuccess)
      err_ = hipMemcpyAsync(dev_ + sent_, stage_[cur_], fill_ * sizeof(double), hipMemcpyHostToDevice,
                            nullptr);
    if (err_ == hipSuccess) err_ = hipEventRecord(ev_[cur_], nullptr);
    sent_ += fill_;
    fill_ = 0;
    cur_ ^= 1;
    if (err_ == hipSuccess && used_[cur_]) err_ = hipEventSynchronize(ev_[cur_]);  // buffer free again
    used_[cur_ ^ 1] = true;
  }
  double* dev_;
  size_t total_;
  double* stage_[2] = {nullptr, nullptr};
  hipEvent_t ev_[2] = {nullptr, nullptr};
  bool used_[2] = {false, false};
  size_t off_ = 0, sent_ = 0, fill_ = 0;
  int cur_ = 0;
  bool overrun_ = false;
  hipError_t err_ = hipSuccess;
};

}  // namespace

// Forward declarations of the pieces of plan construction.
int build_plan(sht_plan_s* P, const sht_plan_opts& o);
int pack_plan(sht_plan_s* P, std::vector<BfTree>& trees);
void free_plan_device(sht_plan_s* P);

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) return _e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EHIP; \
  } while (0)

int build_plan(sht_plan_s* P, const sht_plan_opts& o) {
  const double t0 = now_s();
  const int l = P->l;
  const int L2 = 2 * l;
  const int C = P->C;
  std::vector<double> x(L2), w(L2);
  gauss_legendre(L2, x.data(), w.data());
  P->xp.assign(x.begin() + l, x.end());
  P->wp.assign(w.begin() + l, w.end());
  const int npairs = 2 * L2;
  P->n_pairs = npairs;
  P->n_cols.assign(npairs, 0);
  P->levels.assign(npairs, 0);
  int Lmax = 0;
  std::vector<PairShape> shapes(npairs);
  for (int mp = 0; mp < npairs; ++mp) {
    shapes[mp] = pair_shape(l, C, mp);
    if (P->maps) {  // A^{(m,p)} is n_p x n_p, each pair with its own depth (its finals are its own)
      shapes[mp].rows = shapes[mp].cols;
      shapes[mp].L = butterfly_depth(shapes[mp].cols, C);
    }
    P->n_cols[mp] = shapes[mp].cols;
    P->levels[mp] = shapes[mp].L;
    Lmax = std::max(Lmax, shapes[mp].L);
  }
  P->Lmax = Lmax;

  std::vector<BfTree> trees(npairs);
  // Plan cache: the butterflies of an intact prefix of pairs come from disk; the rest are
  // built below and appended batch by batch (a corrupt or foreign tail is cut off first).
  int nvalid = 0;
  CacheWriter cache;
  if (o.cache_dir) {
    CacheScan scan;
    (void)cache_scan(o.cache_dir, l, P->eps, C, npairs, &shapes, &trees, scan);
    nvalid = scan.valid_pairs;
    P->stats.cache_pairs_loaded = nvalid;
    P->stats.cache_rebuilt = scan.corrupt ? 1 : 0;
    if (nvalid < npairs || scan.corrupt) {
      const int rc = cache.open(o.cache_dir, l, P->eps, C, npairs, scan.corrupt && nvalid == 0 ? 0 : scan.valid_bytes);
      if (rc != SHT_OK) return rc;
    }
  }
  const int nthreads = o.host_threads > 0 ? o.host_threads : host_thread_count();
  double t_cols = 0.0, t_comp = 0.0;
  int err = SHT_OK;
  if (P->maps) {
    // Per-order maps (Section 5): every A^{(m,p)} on the host (its nodes by Sturm bisection
    // and Newton, its rows by the normalized recurrence), one pair per thread, largest first;
    // the leaves then go to the depth-first construction in column order, as for Q^{(m,p)}.
    std::atomic<int> bad{0};
    std::vector<double> tc(npairs, 0.0), ti(npairs, 0.0);
    parallel_for(npairs, nthreads, [&](int mp) {
      if (bad) return;
      try {
        const int n = P->n_cols[mp];
        const double ta = now_s();
        std::vector<double> a(std::max<size_t>(1, static_cast<size_t>(n) * n));
        if (n > 0 && gj_matrix(mp / 2, n, mp % 2, a.data(), n, false) != SHT_OK) {
          bad = SHT_EINTERNAL;
          return;
        }
        const double tb = now_s();
        BfTree& tr = trees[mp];
        tr.init(n, n, C, P->levels[mp], P->eps);
        for (int c = 0; c < (1 << tr.L()); ++c)
          tr.add_leaf(c, a.data() + static_cast<size_t>(std::min(c * C, n)) * n, std::max(n, 1));
        tc[mp] = tb - ta;
        ti[mp] = now_s() - tb;
      } catch (const std::bad_alloc&) {
        bad = SHT_ENOMEM;
      } catch (...) {
        bad = SHT_EINTERNAL;
      }
    });
    if (bad) return bad;
    for (int mp = 0; mp < npairs; ++mp) {  // thread time, per thread
      t_cols += tc[mp] / std::min(nthreads, npairs);
      t_comp += ti[mp] / std::min(nthreads, npairs);
    }
  }
  for (int mp = nvalid; mp < npairs && !P->maps; ++mp)
    trees[mp].init(l, P->n_cols[mp], C, P->levels[mp], P->eps);
  if (!P->maps && o.id_device && nvalid < npairs) {
    CacheAppend append;
    if (cache.is_open())
      append = [&](int first, int end) {
        int rc = SHT_OK;
        for (int mp = first; mp < end && rc == SHT_OK; ++mp) rc = cache.append(mp, trees[mp]);
        return rc == SHT_OK ? cache.flush() : rc;
      };
    try {
      err = build_trees_on_device(P, trees, nvalid, append, t_cols, t_comp);
    } catch (const std::bad_alloc&) {
      err = SHT_ENOMEM;
    } catch (...) {
      err = SHT_EINTERNAL;
    }
  }

  // Device-side column generation, batch by batch.
  const size_t chunk_doubles = static_cast<size_t>(C) * l;
  int batch = static_cast<int>(std::max<size_t>(2, (size_t(64) << 20) / (chunk_doubles * 8)));
  batch = std::min(batch, npairs);
  batch = std::max(2, batch - (batch % 2));

  DevBuf dx, dsw, dm, dp, dn, dprev, dcur, dexp, dout;
  HIP_TRY(dev_alloc(&dx.p, sizeof(double) * l));
  HIP_TRY(dev_alloc(&dsw.p, sizeof(double) * l));
  std::vector<double> sw(l);
  for (int i = 0; i < l; ++i) sw[i] = std::sqrt(2.0 * P->wp[i]);
  HIP_TRY(hipMemcpy(dx.p, P->xp.data(), sizeof(double) * l, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(dsw.p, sw.data(), sizeof(double) * l, hipMemcpyHostToDevice));
  HIP_TRY(dev_alloc(&dm.p, sizeof(int) * batch));
  HIP_TRY(dev_alloc(&dp.p, sizeof(int) * batch));
  HIP_TRY(dev_alloc(&dn.p, sizeof(int) * batch));
  HIP_TRY(dev_alloc(&dprev.p, 2 * sizeof(double) * batch * l));  // double-double state
  HIP_TRY(dev_alloc(&dcur.p, 2 * sizeof(double) * batch * l));
  HIP_TRY(dev_alloc(&dexp.p, sizeof(int) * batch * l));
  HIP_TRY(dev_alloc(&dout.p, sizeof(double) * batch * chunk_doubles));
  double* host_chunk = nullptr;
  HIP_TRY(pinned_alloc(reinterpret_cast<void**>(&host_chunk), sizeof(double) * batch * chunk_doubles));
  std::unique_ptr<double, void (*)(double*)> host_guard(host_chunk,
                                                          [](double* q) { (void)hipHostFree(q); });

  for (int b0 = 0; b0 < npairs && err == SHT_OK && !P->maps && !o.id_device; b0 += batch) {
    const int nb = std::min(batch, npairs - b0);
    if (b0 + nb <= nvalid) continue;  // every butterfly of the batch came from the cache
    std::vector<int> hm(nb), hp(nb), hn(nb);
    int leaves = 0;
    for (int b = 0; b < nb; ++b) {
      hm[b] = (b0 + b) / 2;
      hp[b] = (b0 + b) % 2;
      hn[b] = P->n_cols[b0 + b];
      leaves = std::max(leaves, 1 << P->levels[b0 + b]);
    }
    HIP_TRY(hipMemcpy(dm.p, hm.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dp.p, hp.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dn.p, hn.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
    ColumnBatch cb;
    cb.npairs = nb;
    cb.l = l;
    cb.C = C;
    cb.d_m = static_cast<int*>(dm.p);
    cb.d_p = static_cast<int*>(dp.p);
    cb.d_ncols = static_cast<int*>(dn.p);
    cb.d_prev = static_cast<double*>(dprev.p);
    cb.d_cur = static_cast<double*>(dcur.p);
    cb.d_exp = static_cast<int*>(dexp.p);
    cb.d_out = static_cast<double*>(dout.p);
    cb.d_x = static_cast<const double*>(dx.p);
    cb.d_sw = static_cast<const double*>(dsw.p);
    HIP_TRY(legendre_seed(cb, nullptr));
    for (int c = 0; c < leaves; ++c) {
      double ta = now_s();
      HIP_TRY(legendre_chunk(cb, c, nullptr));
      HIP_TRY(hipMemcpy(host_chunk, dout.p, sizeof(double) * nb * chunk_doubles,
                        hipMemcpyDeviceToHost));
      double tb = now_s();
      t_cols += tb - ta;
      std::atomic<int> bad{0};
      parallel_for(nb, nthreads, [&](int b) {
        BfTree& tr = trees[b0 + b];
        if (b0 + b < nvalid || c >= (1 << tr.L())) return;
        try {
          tr.add_leaf(c, host_chunk + static_cast<size_t>(b) * chunk_doubles, l);
        } catch (const std::bad_alloc&) {
          bad = SHT_ENOMEM;
        } catch (...) {
          bad = SHT_EINTERNAL;
        }
      });
      t_comp += now_s() - tb;
      if (bad) {
        err = bad;
        break;
      }
    }
    if (err == SHT_OK && cache.is_open()) {
      for (int mp = std::max(b0, nvalid); mp < b0 + nb && err == SHT_OK; ++mp) err = cache.append(mp, trees[mp]);
      if (err == SHT_OK) err = cache.flush();
    }
  }
  if (err != SHT_OK) return err;

  // statistics
  sht_stats& st = P->stats;
  st.l = l;
  st.leaf_width = C;
  st.max_levels = Lmax;
  st.eps = P->eps;
  long long nid = 0;
  double sk = 0, sk2 = 0;
  int kmax = 0;
  long long fe = 0, mmax = 0, dense = 0;
  double tmax = 0.0;
  for (auto& t : trees) {
    tmax = std::max(tmax, t.max_abs_t);
    nid += t.n_ids;
    sk += t.sum_k;
    sk2 += t.sum_k2;
    kmax = std::max(kmax, t.k_max);
    fe += t.factor_entries;
    mmax = std::max(mmax, t.m_max_words);
    dense += static_cast<long long>(t.rows()) * t.cols();
  }
  st.n_blocks = nid;
  st.k_max = kmax;
  st.k_avg = nid ? sk / nid : 0.0;
  st.k_sd = nid ? std::sqrt(std::max(0.0, sk2 / nid - st.k_avg * st.k_avg)) : 0.0;
  st.factor_entries = fe;
  st.dense_entries = dense;
  st.m_max_words = mmax;
  st.max_abs_t = tmax;
  st.t_columns_s = t_cols;
  st.t_compress_s = t_comp;
  int rc = pack_plan(P, trees);
  st.t_total_s = now_s() - t0;
  return rc;
}

// ------------------------------------------------------------------------------------------
// packing

int pack_plan(sht_plan_s* P, std::vector<BfTree>& trees) {
  const int l = P->l;
  const int L2 = 2 * l;
  const int npairs = 2 * L2;
  const int Lmax = P->Lmax;
  // Row bases: internal coefficient rows and butterfly vector rows per pair.
  P->in_base.assign(npairs, 0);
  P->v_base.assign(npairs, 0);
  P->v_rows.assign(npairs, 0);
  std::vector<std::vector<std::vector<int>>> voff(npairs);  // [mp][t][block] offsets
  long long in_rows = 0, v_rows = 0;
  for (int mp = 0; mp < npairs; ++mp) {
    P->in_base[mp] = static_cast<int>(in_rows);
    in_rows += P->n_cols[mp];
    const BfTree& T = trees[mp];
    voff[mp].resize(T.L() + 1);
    int vmax = 0;
    for (int t = 0; t <= T.L(); ++t) {
      const int nb = T.nrow(t) * T.ncol(t);
      voff[mp][t].resize(nb + 1);
      int acc = 0;
      for (int b = 0; b < nb; ++b) {
        voff[mp][t][b] = acc;
        acc += T.block(t, b / T.ncol(t), b % T.ncol(t)).k;
      }
      voff[mp][t][nb] = acc;
      vmax = std::max(vmax, acc);
    }
    P->v_base[mp] = static_cast<int>(v_rows);
    P->v_rows[mp] = vmax;
    v_rows += vmax;
  }
  if (in_rows > INT32_MAX || v_rows > INT32_MAX) return SHT_EUNSUPPORTED;
  P->rows_in = in_rows;
  P->rows_v = v_rows;
  P->rows_y = P->maps ? in_rows : static_cast<long long>(L2) * L2;

  // Every T and final S of the trees is packed exactly once (empty ones add nothing), so
  // the pool's size is known before packing starts.
  size_t n_fac_total = 0;
  for (const BfTree& T : trees) n_fac_total += static_cast<size_t>(T.factor_entries);
  {
    const hipError_t ea = dev_alloc(reinterpret_cast<void**>(&P->d.fac),
                                    std::max<size_t>(n_fac_total, 2) * sizeof(double));
    if (ea != hipSuccess) return ea == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EHIP;
  }
  FactorStream fac(P->d.fac, n_fac_total);
  std::vector<uint16_t> idx;
  std::vector<LevelTask> tasks;
  std::vector<FinalTask> finals;
  std::vector<FactorBlock> fblocks;
  P->step_off.assign(Lmax + 1, 0);
  P->step_cnt.assign(Lmax + 1, 0);
  P->step_maxK.assign(Lmax + 1, 0);
  P->step_maxk.assign(Lmax + 1, 0);
  P->step_fac.assign(Lmax + 1, 0.0);
  P->step_rows_in.assign(Lmax + 1, 0.0);
  P->step_rows_out.assign(Lmax + 1, 0.0);
  // Places of every stored matrix in the int8-slice pools (both orientations), filled by
  // sht_plan_prepare; only the offsets are laid out here.
  long long dig_off = 0, dex_off = 0;
  std::vector<I8Block> i8b;
  auto i8_place = [&](int64_t fac_off, int rows, int cols, I8Off& o) {
    o = I8Off{};
    if (rows <= 0 || cols <= 0) return;
    o.dig[0] = dig_off;
    dig_off += i8_tile_bytes(rows, cols);
    o.dig[1] = dig_off;
    dig_off += i8_tile_bytes(cols, rows);
    o.ex[0] = dex_off;
    dex_off += i8_exp_count(rows);
    o.ex[1] = dex_off;
    dex_off += i8_exp_count(cols);
    i8b.push_back({fac_off, rows, cols, o});
  };
  // map (may be null): renumbering of the block's input indices (folded leaves, below)
  auto push_block = [&](const BfBlock& B, int32_t& idx_off, int64_t& fac_off, I8Off& i8o,
                        const std::vector<int>* map) {
    idx_off = static_cast<int32_t>(idx.size());
    for (int v : B.skel) idx.push_back(static_cast<uint16_t>(map ? (*map)[v] : v));
    for (int v : B.red) idx.push_back(static_cast<uint16_t>(map ? (*map)[v] : v));
    fac_off = static_cast<int64_t>(fac.size());
    fac.append(B.T.data(), B.T.size());
    if (!B.T.empty()) fblocks.push_back({fac_off, B.k, B.K - B.k});
    i8_place(fac_off, B.T.empty() ? 0 : B.k, B.K - B.k, i8o);
  };
  // Tasks of a step are independent; they are grouped into size classes (by input length
  // K) so that each class launches with an LDS allocation fitting its own blocks, largest
  // class first.  Factors are packed in launch order so the apply kernels stream them.
  auto kclass = [](int K) { return K <= 96 ? 2 : (K <= 192 ? 1 : 0); };
  struct Proto {
    LevelTask tk;
    const BfBlock* b[2];
    std::vector<int> map;  // folded leaves: level-1 input index -> leaf-pair column
  };
  // Folded leaves.  The columns of Q^{(m,p)} are orthonormal, so every leaf block has full
  // rank and its ID is a pure reordering (k = K, no T): w = x[skel].  For an order with at
  // least one level above the leaves, the level-1 tasks read the coefficients of their two
  // leaves directly (in column order) with their index lists renumbered through the
  // leaves' skeleton orders, and the leaf step is dropped for that order.
  std::vector<char> fold(npairs, 0);
  for (int mp = 0; mp < npairs && !P->maps; ++mp) {  // the order maps read their own input rows
    const BfTree& T = trees[mp];
    if (T.L() < 1) continue;
    bool ident = true;
    for (int c = 0; c < T.ncol(0) && ident; ++c) {
      const BfBlock& B = T.block(0, 0, c);
      ident = B.k == B.K && B.red.empty();  // only the last non-empty leaf can be short
    }
    fold[mp] = ident;
  }
  P->n_folded = 0;
  for (char f : fold) P->n_folded += f;
  P->step_classes.assign(Lmax + 1, {});
  for (int t = 0; t <= Lmax; ++t) {
    P->step_off[t] = static_cast<long long>(tasks.size());
    std::vector<Proto> protos;
    for (int mp = 0; mp < npairs; ++mp) {
      const BfTree& T = trees[mp];
      if (T.L() < t) continue;
      const int vb = P->v_base[mp];
      if (t == 0) {
        if (fold[mp]) continue;
        for (int c = 0; c < T.ncol(0); ++c) {
          const BfBlock& B = T.block(0, 0, c);
          if (B.K == 0) continue;
          Proto pr{};
          pr.tk.in_row = P->in_base[mp] + c * T.C();
          pr.tk.K = B.K;
          pr.tk.out_row[0] = vb + voff[mp][0][c];
          pr.tk.k[0] = B.k;
          pr.tk.k[1] = -1;
          pr.tk.mp = mp;
          pr.b[0] = &B;
          pr.b[1] = nullptr;
          protos.push_back(pr);
        }
      } else {
        const int ncp = T.ncol(t - 1), nc = T.ncol(t);
        for (int q = 0; q < T.nrow(t - 1); ++q) {
          for (int cc = 0; cc < nc; ++cc) {
            const BfBlock& Bt = T.block(t, 2 * q, cc);
            const BfBlock& Bb = T.block(t, 2 * q + 1, cc);
            if (Bt.K == 0) continue;
            Proto pr{};
            pr.tk.in_row = vb + voff[mp][t - 1][q * ncp + 2 * cc];
            pr.tk.K = Bt.K;
            pr.tk.out_row[0] = vb + voff[mp][t][(2 * q) * nc + cc];
            pr.tk.out_row[1] = vb + voff[mp][t][(2 * q + 1) * nc + cc];
            pr.tk.k[0] = Bt.k;
            pr.tk.k[1] = Bb.k;
            pr.tk.mp = -1;
            pr.b[0] = &Bt;
            pr.b[1] = &Bb;
            if (t == 1 && fold[mp]) {
              const BfBlock& Lf = T.block(0, 0, 2 * cc);
              const int kl = Lf.k;
              pr.tk.in_row = P->in_base[mp] + 2 * cc * T.C();
              pr.tk.mp = mp;
              pr.map.resize(Bt.K);
              for (int v = 0; v < Bt.K; ++v)
                pr.map[v] = v < kl ? Lf.skel[v] : Lf.K + T.block(0, 0, 2 * cc + 1).skel[v - kl];
            }
            protos.push_back(pr);
          }
        }
      }
    }
    std::stable_sort(protos.begin(), protos.end(), [&](const Proto& a, const Proto& b) {
      return kclass(a.tk.K) < kclass(b.tk.K);
    });
    for (size_t i = 0; i < protos.size(); ++i) {
      Proto& pr = protos[i];
      LevelTask tk = pr.tk;
      const std::vector<int>* map = pr.map.empty() ? nullptr : &pr.map;
      push_block(*pr.b[0], tk.idx[0], tk.fac[0], tk.i8[0], map);
      int kmx = pr.b[0]->k;
      double nf = static_cast<double>(pr.b[0]->T.size());
      if (pr.b[1]) {
        push_block(*pr.b[1], tk.idx[1], tk.fac[1], tk.i8[1], map);
        kmx = std::max(kmx, pr.b[1]->k);
        nf += static_cast<double>(pr.b[1]->T.size());
      }
      const int cl = kclass(tk.K);
      auto& cls = P->step_classes[t];
      if (cls.empty() || cls.back().cls != cl)
        cls.push_back({static_cast<long long>(tasks.size()) - P->step_off[t], 0, 0, 0, cl});
      cls.back().cnt += 1;
      cls.back().maxK = std::max(cls.back().maxK, tk.K);
      cls.back().maxk = std::max(cls.back().maxk, kmx);
      cls.back().maxnr = std::max(cls.back().maxnr, tk.K - std::min(tk.k[0], tk.k[1] < 0 ? tk.k[0] : tk.k[1]));
      cls.back().fac += nf;
      cls.back().rows_in += tk.K;
      cls.back().rows_out += tk.k[0] + (tk.k[1] > 0 ? tk.k[1] : 0);
      tasks.push_back(tk);
      P->step_maxK[t] = std::max(P->step_maxK[t], tk.K);
      P->step_maxk[t] = std::max(P->step_maxk[t], kmx);
      P->step_fac[t] += nf;
      P->step_rows_in[t] += tk.K;
      P->step_rows_out[t] += tk.k[0] + (tk.k[1] > 0 ? tk.k[1] : 0);
    }
    P->step_cnt[t] = static_cast<long long>(tasks.size()) - P->step_off[t];
  }
  // Final skeleton tasks, grouped like the level tasks by rank (LDS size per launch).
  auto fclass = [](int k) { return k <= 96 ? 1 : 0; };
  struct FProto {
    FinalTask ft;
    const BfFinal* f[2];
  };
  std::vector<FProto> fprotos;
  for (int m = 0; m < L2 && !P->maps; ++m) {
    const BfTree& T0 = trees[2 * m];
    const BfTree& T1 = trees[2 * m + 1];
    const int L = T0.L();
    for (int r = 0; r < (1 << L); ++r) {
      FProto pr{};
      FinalTask& ft = pr.ft;
      ft.m = m;
      ft.row0 = T0.row_lo(L, r);
      ft.h = T0.row_h(L, r);
      ft.vbuf = L % 2;
      for (int p = 0; p < 2; ++p) {
        const BfTree& T = p ? T1 : T0;
        pr.f[p] = &T.final_block(r);
        ft.k[p] = pr.f[p]->k;
        ft.in_row[p] = P->v_base[2 * m + p] + voff[2 * m + p][L][r];
      }
      if (ft.h > 0) fprotos.push_back(pr);
    }
  }
  std::stable_sort(fprotos.begin(), fprotos.end(), [&](const FProto& a, const FProto& b) {
    return fclass(std::max(a.ft.k[0], a.ft.k[1])) < fclass(std::max(b.ft.k[0], b.ft.k[1]));
  });
  P->final_classes.clear();
  for (FProto& pr : fprotos) {
    FinalTask ft = pr.ft;
    for (int p = 0; p < 2; ++p) {
      const BfFinal& f = *pr.f[p];
      ft.fac[p] = static_cast<int64_t>(fac.size());
      fac.append(f.S.data(), f.S.size());
      if (!f.S.empty()) fblocks.push_back({ft.fac[p], f.h, f.k});
      i8_place(ft.fac[p], f.S.empty() ? 0 : f.h, f.k, ft.i8[p]);
    }
    const int kmx = std::max(ft.k[0], ft.k[1]);
    const int cl = fclass(kmx);
    if (P->final_classes.empty() || P->final_classes.back().cls != cl)
      P->final_classes.push_back({static_cast<long long>(finals.size()), 0, 0, 0, cl});
    P->final_classes.back().cnt += 1;
    P->final_classes.back().maxK = std::max(P->final_classes.back().maxK, ft.h);
    P->final_classes.back().maxk = std::max(P->final_classes.back().maxk, kmx);
    P->final_classes.back().maxnr = std::max(P->final_classes.back().maxnr, kmx);
    P->final_classes.back().fac += static_cast<double>(ft.h) * (ft.k[0] + ft.k[1]);
    P->final_classes.back().rows_in += ft.k[0] + ft.k[1];
    P->final_classes.back().rows_out += 2.0 * ft.h;
    finals.push_back(ft);
    P->final_fac += static_cast<double>(ft.h) * (ft.k[0] + ft.k[1]);
    P->final_rows_v += ft.k[0] + ft.k[1];
    P->final_rows_y += 2.0 * ft.h;
    P->final_maxh = std::max(P->final_maxh, ft.h);
    P->final_maxk = std::max(P->final_maxk, kmx);
  }
  // Per-order maps: one final per (pair, row node), written straight to its output rows.
  std::vector<OrderFinal> ofinals;
  for (int mp = 0; mp < npairs && P->maps; ++mp) {
    const BfTree& T = trees[mp];
    const int L = T.L();
    for (int r = 0; r < (1 << L); ++r) {
      const BfFinal& f = T.final_block(r);
      if (f.h <= 0) continue;
      OrderFinal of{};
      of.in_row = P->v_base[mp] + voff[mp][L][r];
      of.out_row = P->in_base[mp] + f.row0;
      of.h = f.h;
      of.k = f.k;
      of.vbuf = L % 2;
      of.fac = static_cast<int64_t>(fac.size());
      fac.append(f.S.data(), f.S.size());
      I8Off unused;
      if (!f.S.empty()) fblocks.push_back({of.fac, f.h, f.k});
      i8_place(of.fac, f.S.empty() ? 0 : f.h, f.k, unused);
      ofinals.push_back(of);
      P->final_fac += static_cast<double>(f.h) * f.k;
      P->final_rows_v += f.k;
      P->final_rows_y += f.h;
      P->ofinal_maxk = std::max(P->ofinal_maxk, f.k);
      P->ofinal_maxh = std::max(P->ofinal_maxh, f.h);
    }
  }
  P->n_ofinal = static_cast<long long>(ofinals.size());
  P->n_final = static_cast<long long>(finals.size());
  P->n_fac = static_cast<long long>(fac.size());
  P->n_dig = dig_off;
  P->n_dex = dex_off;
  P->n_idx = static_cast<long long>(idx.size());
  {
    const int rc = fac.close();
    if (rc != SHT_OK) return rc;
  }
  // free host trees early
  std::vector<BfTree>().swap(trees);

  // device upload
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) bytes = 16;
    hipError_t e = dev_alloc(dst, bytes);
    if (e != hipSuccess) return e;
    if (src) return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return hipSuccess;
  };
  std::vector<double> invD(l), D(l);
  for (int i = 0; i < l; ++i) {
    D[i] = std::sqrt(2.0 * P->wp[i]);
    invD[i] = 1.0 / D[i];
  }
  const int N = 4 * l;
  std::vector<double> tw(2 * static_cast<size_t>(N));
  for (int q = 0; q < N; ++q) {
    const long double ang = 2.0L * 3.141592653589793238462643383279502884L * q / N;
    tw[2 * q] = static_cast<double>(cosl(ang));
    tw[2 * q + 1] = static_cast<double>(sinl(ang));
  }
  std::vector<PairDesc> pd(npairs);
  for (int mp = 0; mp < npairs; ++mp) {
    pd[mp].m = mp / 2;
    pd[mp].p = mp % 2;
    pd[mp].n = P->n_cols[mp];
    pd[mp].in_base = P->in_base[mp];
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.idx), idx.data(), idx.size() * sizeof(uint16_t));
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.tasks), tasks.data(), tasks.size() * sizeof(LevelTask));
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.finals), finals.data(), finals.size() * sizeof(FinalTask));
  if (e == hipSuccess)
    e = up(reinterpret_cast<void**>(&P->d.ofinals), ofinals.data(), ofinals.size() * sizeof(OrderFinal));
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.pairs), pd.data(), pd.size() * sizeof(PairDesc));
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.invD), invD.data(), invD.size() * sizeof(double));
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.D), D.data(), D.size() * sizeof(double));
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.twiddle), tw.data(), tw.size() * sizeof(double));
  // transposed copies for the analysis direction, built on the device
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&P->d.fac_t), nullptr, n_fac_total * sizeof(double));
  FactorBlock* dblocks = nullptr;
  if (e == hipSuccess) e = up(reinterpret_cast<void**>(&dblocks), fblocks.data(), fblocks.size() * sizeof(FactorBlock));
  if (e == hipSuccess)
    e = transpose_factors(P->d.fac, P->d.fac_t, dblocks, static_cast<long long>(fblocks.size()), nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  P->d.blocks = dblocks;  // kept: the split copies are derived from it on first use
  P->n_blocks = static_cast<long long>(fblocks.size());
  if (e == hipSuccess && i8b.size() != fblocks.size()) return SHT_EINTERNAL;
  if (e == hipSuccess)
    e = up(reinterpret_cast<void**>(&P->d.i8blocks), i8b.data(), i8b.size() * sizeof(I8Block));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EHIP;
  P->stats.device_bytes =
      static_cast<long long>(2 * n_fac_total * 8 + idx.size() * 2 + tasks.size() * sizeof(LevelTask) +
                             finals.size() * sizeof(FinalTask) + ofinals.size() * sizeof(OrderFinal) +
                             pd.size() * sizeof(PairDesc) +
                             (invD.size() + D.size() + tw.size()) * 8);
  return SHT_OK;
}

void free_plan_device(sht_plan_s* P) {
  void* ptrs[] = {P->d.fac,    P->d.fac_t,   P->d.fac_hl, P->d.fac_t_hl, P->d.dig,
                  P->d.dex,    P->d.i8blocks, P->d.blocks, P->d.idx,     P->d.tasks,
                  P->d.finals, P->d.ofinals, P->d.pairs,  P->d.invD,     P->d.D,
                  P->d.twiddle};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  P->d = DeviceFactors{};
}

}  // namespace sht
