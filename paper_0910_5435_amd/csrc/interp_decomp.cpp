// Host FP64 precompute: interpolative decompositions and the depth-first
// butterfly construction.
//
// ID (Section 3.1, Remark QR_algorithm): Householder QR with column pivoting
// (largest remaining column norm, lowest index on ties).  After k steps
// A P = Q [R11 R12; 0 R22]; the skeleton is the first k pivots and
// T = R11^{-1} R12 gives A[:, red] ~= A[:, skel] T with error ||R22||.  The rank
// is the least k with ||R22||_F <= eps (Remark adaptivity; the rank property of
// Section 3.2 measures blocks in the Frobenius norm).  Exchanges of skeleton and
// redundant columns then bring every |T_ij| to at most 2, as the Remark requires.
//
// Butterfly (Section 3.2, equations (1)-(6), (top), (bottom)) built depth-first
// (Section 4): only the skeleton columns of unprocessed blocks are kept between
// merges, so a column chunk is needed once and then dropped.
#include "interp_decomp.h"

#include <sched.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace sht {

int host_thread_count() {
  int n = static_cast<int>(std::max(1u, std::thread::hardware_concurrency()));
  cpu_set_t set;
  if (sched_getaffinity(0, sizeof set, &set) == 0) n = std::max(1, CPU_COUNT(&set));
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {
    const int cap = std::atoi(e);
    if (cap > 0) n = std::min(n, cap);
  }
  return n;
}

namespace {

// sum_i a[i] b[i] over 16 independent partial sums combined pairwise: a single running
// sum would be one dependent add chain, which bounds the QR below by add latency.
double dot(const double* a, const double* b, int n) {
  double s[16] = {};
  int i = 0;
  for (; i + 16 <= n; i += 16)
    for (int u = 0; u < 16; ++u) s[u] += a[i + u] * b[i + u];
  for (int u = 0; i < n; ++i, ++u) s[u] += a[i] * b[i];
  for (int w = 8; w > 0; w /= 2)
    for (int u = 0; u < w; ++u) s[u] += s[u + w];
  return s[0];
}

// b -= c a
void axpy(double c, const double* a, double* b, int n) {
  for (int i = 0; i < n; ++i) b[i] -= c * a[i];
}

// The reflector v applied to four columns at once (v is read once per pass):
// c_q -= tau (c_q[0] + v . c_q[1:]) [1; v] with v = col[1:].
typedef double d4 __attribute__((ext_vector_type(4)));
inline d4 ld4(const double* p) {
  d4 v;
  std::memcpy(&v, p, sizeof v);
  return v;
}
inline void st4(double* p, d4 v) { std::memcpy(p, &v, sizeof v); }

void reflect4(double tau, const double* col, double* const c[4], int n) {
  d4 s0[4] = {}, s1[4] = {};
  int i = 1;
  for (; i + 8 <= n; i += 8) {
    const d4 v0 = ld4(col + i), v1 = ld4(col + i + 4);
    for (int q = 0; q < 4; ++q) {
      s0[q] += v0 * ld4(c[q] + i);
      s1[q] += v1 * ld4(c[q] + i + 4);
    }
  }
  double d[4];
  for (int q = 0; q < 4; ++q) {
    const d4 t = s0[q] + s1[q];
    double r = (t.x + t.z) + (t.y + t.w);
    for (int e = i; e < n; ++e) r += col[e] * c[q][e];
    d[q] = tau * (c[q][0] + r);
    c[q][0] -= d[q];
  }
  i = 1;
  for (; i + 4 <= n; i += 4) {
    const d4 v = ld4(col + i);
    for (int q = 0; q < 4; ++q) st4(c[q] + i, ld4(c[q] + i) - d[q] * v);
  }
  for (; i < n; ++i)
    for (int q = 0; q < 4; ++q) c[q][i] -= d[q] * col[i];
}

// One Householder step on the m x n column-major a at column s: the reflector
// H = I - tau v v^T with v = [1; a[s+1:, s]] zeroes a[s+1:, s] (v is kept there, the new
// diagonal entry at a[s, s]) and is applied to columns s+1 .. n-1.
void householder_step(double* a, int m, int n, int s) {
  double* col = a + static_cast<size_t>(s) * m;
  const double alpha = col[s];
  const double xn2 = dot(col + s + 1, col + s + 1, m - s - 1);
  if (!(xn2 > 0.0)) return;  // already upper triangular in this column: H = I
  const double beta = -std::copysign(std::sqrt(alpha * alpha + xn2), alpha);
  const double tau = (beta - alpha) / beta;
  const double scale = 1.0 / (alpha - beta);
  for (int i = s + 1; i < m; ++i) col[i] *= scale;
  col[s] = beta;
  int j = s + 1;
  for (; j + 4 <= n; j += 4) {
    double* const c4[4] = {a + static_cast<size_t>(j) * m + s, a + static_cast<size_t>(j + 1) * m + s,
                           a + static_cast<size_t>(j + 2) * m + s, a + static_cast<size_t>(j + 3) * m + s};
    reflect4(tau, col + s, c4, m - s);
  }
  for (; j < n; ++j) {
    double* cj = a + static_cast<size_t>(j) * m;
    const double d = tau * (cj[s] + dot(col + s + 1, cj + s + 1, m - s - 1));
    cj[s] -= d;
    axpy(d, col + s + 1, cj + s + 1, m - s - 1);
  }
}

// T = R11^{-1} R12 (k x (n - k), column-major) from the triangular factor held in the
// first k rows of a, by back substitution one column at a time; once t[i] is known its
// multiple of column i of R11 leaves the rows above (contiguous access).  Returns max |T|.
double solve_t(const double* a, int m, int n, int k, std::vector<double>& T) {
  const int nr = n - k;
  T.assign(static_cast<size_t>(k) * nr, 0.0);
  double mx = 0.0;
  for (int j = 0; j < nr; ++j) {
    double* t = T.data() + static_cast<size_t>(j) * k;
    std::memcpy(t, a + static_cast<size_t>(k + j) * m, sizeof(double) * k);
    for (int i = k - 1; i >= 0; --i) {
      const double* ri = a + static_cast<size_t>(i) * m;
      t[i] /= ri[i];
      axpy(t[i], ri, t, i);
      mx = std::max(mx, std::fabs(t[i]));
    }
  }
  return mx;
}

}  // namespace

void interp_decomp(const double* A, int m, int n, int lda, double eps, IdResult& out,
                   IdWork& w) {
  out.k = 0;
  out.skel.clear();
  out.red.clear();
  out.T.clear();
  out.max_abs_t = 0.0;
  if (n <= 0) return;
  if (m <= 0) {
    out.red.resize(n);
    std::iota(out.red.begin(), out.red.end(), 0);
    return;
  }
  w.a.resize(static_cast<size_t>(m) * n);
  for (int j = 0; j < n; ++j)
    std::memcpy(&w.a[static_cast<size_t>(j) * m], A + static_cast<size_t>(j) * lda,
                sizeof(double) * m);
  double* a = w.a.data();
  w.perm.resize(n);
  std::iota(w.perm.begin(), w.perm.end(), 0);
  w.nrm.assign(n, 0.0);
  w.nrm0.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double* c = a + static_cast<size_t>(j) * m;
    w.nrm[j] = w.nrm0[j] = dot(c, c, m);
  }
  const int kmax = std::min(m, n);
  const double eps2 = eps * eps;
  int s = 0;
  for (; s < kmax; ++s) {
    double resid = 0.0;
    int p = s;
    for (int j = s; j < n; ++j) {
      resid += w.nrm[j];
      if (w.nrm[j] > w.nrm[p]) p = j;
    }
    if (resid <= eps2) break;
    if (p != s) {
      double* cs = a + static_cast<size_t>(s) * m;
      double* cp = a + static_cast<size_t>(p) * m;
      for (int i = 0; i < m; ++i) std::swap(cs[i], cp[i]);
      std::swap(w.perm[s], w.perm[p]);
      std::swap(w.nrm[s], w.nrm[p]);
      std::swap(w.nrm0[s], w.nrm0[p]);
    }
    householder_step(a, m, n, s);
    for (int j = s + 1; j < n; ++j) {
      const double* cj = a + static_cast<size_t>(j) * m;
      // Downdate the trailing column norm; recompute it exactly once the
      // downdated value has lost too many digits to cancellation.
      double nv = w.nrm[j] - cj[s] * cj[s];
      if (nv < 1e-6 * w.nrm0[j]) {
        nv = dot(cj + s + 1, cj + s + 1, m - s - 1);
        w.nrm0[j] = nv;
      }
      w.nrm[j] = nv;
    }
    w.nrm[s] = 0.0;
  }
  const int k = s;
  out.k = k;
  out.max_abs_t = solve_t(a, m, n, k, out.T);
  // Remark QR_algorithm asks for interpolation coefficients of magnitude at most 2, which
  // column pivoting nearly always gives.  Where it does not, the skeleton column i and the
  // redundant column j of the largest |T_ij| > 2 are exchanged (the Gu-Eisenstat step:
  // |det R11| grows by |T_ij| each time, so no exchange repeats), and the block is factored
  // again without pivoting in the new order.  An exchange whose residual ||R22||_F would
  // exceed eps is not taken.
  for (int it = 0; it < 64 && k > 0 && k < n && out.max_abs_t > 2.0; ++it) {
    size_t arg = 0;
    for (size_t q = 1; q < out.T.size(); ++q)
      if (std::fabs(out.T[q]) > std::fabs(out.T[arg])) arg = q;
    const int i = static_cast<int>(arg % k), j = static_cast<int>(arg / k);
    w.trial = w.perm;
    std::swap(w.trial[i], w.trial[k + j]);
    w.b.resize(static_cast<size_t>(m) * n);
    for (int c = 0; c < n; ++c)
      std::memcpy(&w.b[static_cast<size_t>(c) * m], A + static_cast<size_t>(w.trial[c]) * lda,
                  sizeof(double) * m);
    for (int q = 0; q < k; ++q) householder_step(w.b.data(), m, n, q);
    double resid = 0.0;
    for (int c = k; c < n; ++c) {
      const double* col = w.b.data() + static_cast<size_t>(c) * m;
      resid += dot(col + k, col + k, m - k);
    }
    if (resid > eps2) break;
    w.perm.swap(w.trial);
    w.a.swap(w.b);
    a = w.a.data();
    out.max_abs_t = solve_t(a, m, n, k, out.T);
  }
  out.skel.assign(w.perm.begin(), w.perm.begin() + k);
  out.red.assign(w.perm.begin() + k, w.perm.end());
}

int butterfly_depth(int cols, int C) {
  int leaves = (cols + C - 1) / C;
  int L = 0;
  while ((1 << L) < leaves) ++L;
  return L;
}

void BfTree::init(int rows, int cols, int C, int L, double eps) {
  if (rows < 0 || cols < 0 || C < 1 || L < 0 || L > 24)
    throw std::invalid_argument("BfTree::init: bad shape");
  if ((1 << L) * static_cast<long long>(C) < cols)
    throw std::invalid_argument("BfTree::init: leaves do not cover the columns");
  if (rows > 0 && (1 << L) > rows)
    throw std::invalid_argument("BfTree::init: more row blocks than rows");
  rows_ = rows;
  cols_ = cols;
  C_ = C;
  L_ = L;
  eps_ = eps;
  next_leaf_ = 0;
  row_lo_.assign(L + 1, {});
  row_h_.assign(L + 1, {});
  row_lo_[0] = {0};
  row_h_[0] = {rows};
  for (int t = 1; t <= L; ++t) {
    row_lo_[t].resize(1 << t);
    row_h_[t].resize(1 << t);
    for (int q = 0; q < (1 << (t - 1)); ++q) {
      const int lo = row_lo_[t - 1][q], h = row_h_[t - 1][q];
      const int top = (h + 1) / 2;
      row_lo_[t][2 * q] = lo;
      row_h_[t][2 * q] = top;
      row_lo_[t][2 * q + 1] = lo + top;
      row_h_[t][2 * q + 1] = h - top;
    }
  }
  blocks_.assign(L + 1, {});
  pending_.assign(L + 1, {});
  for (int t = 0; t <= L; ++t) {
    blocks_[t].assign(static_cast<size_t>(nrow(t)) * ncol(t), BfBlock{});
    pending_[t].assign(static_cast<size_t>(nrow(t)) * ncol(t), Pending{});
  }
  finals_.assign(1 << L, BfFinal{});
  k_max = 0;
  n_ids = 0;
  sum_k = sum_k2 = 0.0;
  factor_entries = 0;
  words_now = m_max_words = 0;
  max_abs_t = 0.0;
}

int BfTree::leaf_width(int c) const {
  long long lo = static_cast<long long>(c) * C_;
  long long w = std::min<long long>(C_, cols_ - lo);
  return w > 0 ? static_cast<int>(w) : 0;
}

void BfTree::record(IdResult& id, int h, int K, BfBlock& blk, bool take) {
  blk.k = id.k;
  blk.K = K;
  if (take) {
    blk.skel = std::move(id.skel);
    blk.red = std::move(id.red);
    blk.T = std::move(id.T);
  } else {
    blk.skel = id.skel;
    blk.red = id.red;
    blk.T = id.T;
  }
  max_abs_t = std::max(max_abs_t, id.max_abs_t);
  factor_entries += static_cast<long long>(blk.T.size());
  k_max = std::max(k_max, blk.k);
  if (K > 0) {  // rank statistics over the blocks that exist (a padded tree has empty slots)
    n_ids += 1;
    sum_k += blk.k;
    sum_k2 += static_cast<double>(blk.k) * blk.k;
  }
  words_now += static_cast<long long>(h) * blk.k;  // the block's pending skeleton columns
}

void BfTree::assemble(std::vector<std::vector<IdResult>>& ids, std::vector<std::vector<double>>& S,
                      std::vector<std::vector<int>>& cols) {
  if (static_cast<int>(ids.size()) != L_ + 1 || static_cast<int>(S.size()) != (1 << L_) ||
      static_cast<int>(cols.size()) != (1 << L_))
    throw std::invalid_argument("BfTree::assemble: shape");
  for (int t = 0; t <= L_; ++t)
    if (ids[t].size() != blocks_[t].size()) throw std::invalid_argument("BfTree::assemble: shape");
  // the depth-first order of add_leaf and merge, with the IDs given instead of computed
  for (int c = 0; c < (1 << L_); ++c) {
    const int width = leaf_width(c);
    const long long chunk_words = static_cast<long long>(rows_) * width;
    m_max_words = std::max(m_max_words, words_now + chunk_words);
    IdResult& id = ids[0][c];
    if (static_cast<int>(id.skel.size() + id.red.size()) != width)
      throw std::invalid_argument("BfTree::assemble: leaf ID");
    record(id, rows_, width, blocks_[0][c], true);
    m_max_words = std::max(m_max_words, words_now + chunk_words);
    for (int t = 1; t <= L_ && ((c + 1) % (1 << t)) == 0; ++t) {
      const int cc = c >> t;
      for (int q = 0; q < nrow(t - 1); ++q) {
        const int ncp = ncol(t - 1);
        const int h = row_h_[t - 1][q];
        const int kL = blocks_[t - 1][q * ncp + 2 * cc].k, kR = blocks_[t - 1][q * ncp + 2 * cc + 1].k;
        const int K = kL + kR;
        for (int half = 0; half < 2; ++half) {
          const int r = 2 * q + half;
          IdResult& m = ids[t][r * ncol(t) + cc];
          if (static_cast<int>(m.skel.size() + m.red.size()) != K)
            throw std::invalid_argument("BfTree::assemble: merged ID");
          record(m, row_h_[t][r], K, blocks_[t][r * ncol(t) + cc], true);
          m_max_words = std::max(m_max_words, words_now + static_cast<long long>(h) * K);
        }
        words_now -= static_cast<long long>(h) * K;
      }
    }
  }
  next_leaf_ = 1 << L_;
  for (int r = 0; r < (1 << L_); ++r) {
    BfFinal& f = finals_[r];
    f.row0 = row_lo_[L_][r];
    f.h = row_h_[L_][r];
    f.k = blocks_[L_][r].k;
    if (static_cast<int>(cols[r].size()) != f.k || static_cast<long long>(S[r].size()) != static_cast<long long>(f.h) * f.k)
      throw std::invalid_argument("BfTree::assemble: final skeleton");
    f.S = std::move(S[r]);
    f.cols = std::move(cols[r]);
    factor_entries += static_cast<long long>(f.S.size());
  }
}

void BfTree::id_into(const double* a, int h, int K, int lda, BfBlock& blk, Pending& pend,
                     const int* gcols) {
  interp_decomp(a, h, K, lda, eps_, id_, work_);
  record(id_, h, K, blk);
  pend.vals.resize(static_cast<size_t>(h) * blk.k);
  pend.gcols.resize(blk.k);
  for (int q = 0; q < blk.k; ++q) {
    const int src = blk.skel[q];
    std::memcpy(&pend.vals[static_cast<size_t>(q) * h], a + static_cast<size_t>(src) * lda,
                sizeof(double) * h);
    pend.gcols[q] = gcols[src];
  }
  pend.live = true;
}

void BfTree::add_leaf(int c, const double* chunk, int ld) {
  if (c != next_leaf_) throw std::logic_error("BfTree::add_leaf: leaves must come in order");
  const int width = leaf_width(c);
  // the chunk itself is matrix storage held during this step
  const long long chunk_words = static_cast<long long>(rows_) * width;
  m_max_words = std::max(m_max_words, words_now + chunk_words);
  std::vector<int> gcols(width);
  for (int j = 0; j < width; ++j) gcols[j] = c * C_ + j;
  id_into(chunk, rows_, width, ld, blocks_[0][c], pending_[0][c], gcols.data());
  m_max_words = std::max(m_max_words, words_now + chunk_words);
  ++next_leaf_;
  // Merge as far as the leaves constructed so far allow (depth-first order).
  for (int t = 1; t <= L_ && ((c + 1) % (1 << t)) == 0; ++t) merge(t, c >> t);
  if (complete()) {
    for (int r = 0; r < (1 << L_); ++r) {
      Pending& p = pending_[L_][r * ncol(L_) + 0];
      BfFinal& f = finals_[r];
      f.row0 = row_lo_[L_][r];
      f.h = row_h_[L_][r];
      f.k = blocks_[L_][r].k;
      f.S = p.vals;
      f.cols = p.gcols;
      factor_entries += static_cast<long long>(f.S.size());
    }
  }
}

void BfTree::merge(int t, int cc) {
  // Blocks (t-1, q, 2cc) | (t-1, q, 2cc+1) on the rows of node q are concatenated
  // and split into top (2q) and bottom (2q+1) halves; each half is recompressed.
  for (int q = 0; q < nrow(t - 1); ++q) {
    const int ncp = ncol(t - 1);
    Pending& PL = pending_[t - 1][q * ncp + 2 * cc];
    Pending& PR = pending_[t - 1][q * ncp + 2 * cc + 1];
    const int h = row_h_[t - 1][q];
    const int kL = static_cast<int>(PL.gcols.size());
    const int kR = static_cast<int>(PR.gcols.size());
    const int K = kL + kR;
    scratch_.resize(static_cast<size_t>(h) * K);
    if (kL) std::memcpy(scratch_.data(), PL.vals.data(), sizeof(double) * h * kL);
    if (kR)
      std::memcpy(scratch_.data() + static_cast<size_t>(h) * kL, PR.vals.data(),
                  sizeof(double) * h * kR);
    std::vector<int> gc(K);
    for (int j = 0; j < kL; ++j) gc[j] = PL.gcols[j];
    for (int j = 0; j < kR; ++j) gc[kL + j] = PR.gcols[j];
    const long long freed = static_cast<long long>(PL.vals.size() + PR.vals.size());
    for (int half = 0; half < 2; ++half) {
      const int r = 2 * q + half;
      const int off = row_lo_[t][r] - row_lo_[t - 1][q];
      const int hh = row_h_[t][r];
      id_into(scratch_.data() + off, hh, K, h, blocks_[t][r * ncol(t) + cc],
              pending_[t][r * ncol(t) + cc], gc.data());
      m_max_words = std::max(m_max_words, words_now + static_cast<long long>(h) * K);
    }
    words_now -= freed;
    std::vector<double>().swap(PL.vals);
    std::vector<double>().swap(PR.vals);
    PL.live = PR.live = false;
  }
}

// ------------------------------------------------------------------ serialisation
namespace {

class ByteWriter {
 public:
  explicit ByteWriter(std::vector<unsigned char>& out) : out_(out) {}
  template <typename T>
  void put(const T& v) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
    out_.insert(out_.end(), b, b + sizeof(T));
  }
  template <typename T>
  void put_vec(const std::vector<T>& v) {
    put(static_cast<uint64_t>(v.size()));
    const unsigned char* b = reinterpret_cast<const unsigned char*>(v.data());
    out_.insert(out_.end(), b, b + v.size() * sizeof(T));
  }

 private:
  std::vector<unsigned char>& out_;
};

class ByteReader {
 public:
  ByteReader(const unsigned char* p, size_t n) : p_(p), n_(n) {}
  template <typename T>
  bool get(T& v) {
    if (n_ - off_ < sizeof(T)) return false;
    std::memcpy(&v, p_ + off_, sizeof(T));
    off_ += sizeof(T);
    return true;
  }
  template <typename T>
  bool get_vec(std::vector<T>& v, uint64_t max_count) {
    uint64_t c = 0;
    if (!get(c) || c > max_count || (n_ - off_) / sizeof(T) < c) return false;
    v.resize(c);
    std::memcpy(v.data(), p_ + off_, c * sizeof(T));
    off_ += c * sizeof(T);
    return true;
  }
  bool done() const { return off_ == n_; }

 private:
  const unsigned char* p_;
  size_t n_, off_ = 0;
};

}  // namespace

void BfTree::save(std::vector<unsigned char>& out) const {
  ByteWriter w(out);
  w.put(static_cast<int32_t>(rows_));
  w.put(static_cast<int32_t>(cols_));
  w.put(static_cast<int32_t>(C_));
  w.put(static_cast<int32_t>(L_));
  w.put(eps_);
  w.put(static_cast<int32_t>(k_max));
  w.put(static_cast<int64_t>(n_ids));
  w.put(sum_k);
  w.put(sum_k2);
  w.put(static_cast<int64_t>(factor_entries));
  w.put(static_cast<int64_t>(m_max_words));
  w.put(max_abs_t);
  for (int t = 0; t <= L_; ++t)
    for (const BfBlock& b : blocks_[t]) {
      w.put(static_cast<int32_t>(b.k));
      w.put(static_cast<int32_t>(b.K));
      w.put_vec(b.skel);
      w.put_vec(b.red);
      w.put_vec(b.T);
    }
  for (const BfFinal& f : finals_) {
    w.put(static_cast<int32_t>(f.row0));
    w.put(static_cast<int32_t>(f.h));
    w.put(static_cast<int32_t>(f.k));
    w.put_vec(f.S);
    w.put_vec(f.cols);
  }
}

bool BfTree::load(const unsigned char* p, size_t n, int rows, int cols, int C, int L, double eps) {
  ByteReader r(p, n);
  int32_t rr = 0, cc = 0, c = 0, l = 0, km = 0;
  double e = 0.0;
  int64_t nid = 0, fe = 0, mw = 0;
  if (!r.get(rr) || !r.get(cc) || !r.get(c) || !r.get(l) || !r.get(e)) return false;
  if (rr != rows || cc != cols || c != C || l != L || e != eps) return false;
  init(rows, cols, C, L, eps);
  if (!r.get(km) || !r.get(nid) || !r.get(sum_k) || !r.get(sum_k2) || !r.get(fe) || !r.get(mw) || !r.get(max_abs_t))
    return false;
  k_max = km;
  n_ids = nid;
  factor_entries = fe;
  m_max_words = mw;
  const uint64_t cap = static_cast<uint64_t>(rows + 1) * (cols + 1) + 16;
  long long entries = 0;
  for (int t = 0; t <= L_; ++t)
    for (BfBlock& b : blocks_[t]) {
      int32_t k = 0, K = 0;
      if (!r.get(k) || !r.get(K) || !r.get_vec(b.skel, cap) || !r.get_vec(b.red, cap) || !r.get_vec(b.T, cap))
        return false;
      b.k = k;
      b.K = K;
      if (k < 0 || K < k || b.skel.size() != static_cast<size_t>(k) || b.red.size() != static_cast<size_t>(K - k) ||
          (!b.T.empty() && b.T.size() != static_cast<size_t>(k) * (K - k)))
        return false;
      for (int v : b.skel)
        if (v < 0 || v >= K) return false;
      for (int v : b.red)
        if (v < 0 || v >= K) return false;
      entries += static_cast<long long>(b.T.size());
    }
  for (int q = 0; q < (1 << L_); ++q) {
    BfFinal& f = finals_[q];
    int32_t row0 = 0, h = 0, k = 0;
    if (!r.get(row0) || !r.get(h) || !r.get(k) || !r.get_vec(f.S, cap) || !r.get_vec(f.cols, cap)) return false;
    f.row0 = row0;
    f.h = h;
    f.k = k;
    if (row0 != row_lo_[L_][q] || h != row_h_[L_][q] || k < 0 || f.cols.size() != static_cast<size_t>(k) ||
        (!f.S.empty() && f.S.size() != static_cast<size_t>(h) * k))
      return false;
    entries += static_cast<long long>(f.S.size());
  }
  if (entries != factor_entries || !r.done()) return false;
  next_leaf_ = 1 << L_;  // complete: no pending state
  return true;
}

}  // namespace sht
