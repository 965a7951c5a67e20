// Interpolative decomposition by column-pivoted Householder QR (Section 3.1,
// Lemma interpolation_lemma and Remark QR_algorithm), and the multilevel
// butterfly representation built by the depth-first traversal of Section 4.
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace sht {

// A[:, red] ~= A[:, skel] * T  with T = R11^{-1} R12 (k x (n-k), column-major:
// T[j * k + i]).  The interpolation matrix of the paper has the identity at the
// skeleton columns and T at the redundant ones.
struct IdResult {
  int k = 0;
  std::vector<int> skel;
  std::vector<int> red;
  std::vector<double> T;
  double max_abs_t = 0.0;
};

// Threads for the host precompute when the caller leaves the count to the library: the
// CPUs this process may run on, capped by OMP_NUM_THREADS when that is set to a positive
// number (a container's CPU quota does not show in the affinity mask).
int host_thread_count();

struct IdWork {
  std::vector<double> a, b;  // the block being factored; b: a refactoring after an exchange
  std::vector<double> nrm, nrm0;
  std::vector<int> perm, trial;
};

// Rank chosen adaptively (Remark adaptivity): the least k whose residual block
// R22 of the pivoted QR has Frobenius norm <= eps; skeleton exchanges then bound
// |T| by 2 (Remark QR_algorithm) without giving up that residual bound.  a is
// rows x cols, column-major with leading dimension lda.
void interp_decomp(const double* a, int rows, int cols, int lda, double eps, IdResult& out,
                   IdWork& work);

// One ID of the butterfly: output w = in[skel] + T in[red] (synthesis) or its transpose.
struct BfBlock {
  int k = 0;
  int K = 0;
  std::vector<int> skel, red;
  std::vector<double> T;
};

// Skeleton columns of a level-L block restricted to its rows (the final factor).
struct BfFinal {
  int row0 = 0, h = 0, k = 0;
  std::vector<double> S;  // h x k column-major
  std::vector<int> cols;  // global column indices
};

// Butterfly of an rows x cols matrix with leaf width C and depth L.  Level t
// (0 = leaves) holds 2^t row nodes times 2^(L-t) column nodes; row node r of
// level t splits into 2r (first ceil(h/2) rows) and 2r+1 at level t+1.
class BfTree {
 public:
  BfTree() = default;
  void init(int rows, int cols, int C, int L, double eps);
  // Depth-first traversal (Section 4): leaf c is constructed only after every
  // merge its left neighbours allow has been done.  `leaf` must fill a
  // rows x width column-major array with columns [c*C, c*C + width).
  void add_leaf(int c, const double* chunk, int ld);
  bool complete() const { return next_leaf_ == (1 << L_); }
  // The same tree from IDs computed elsewhere (the device builder): ids[t][r * ncol(t) + c]
  // for every block (IdResult as interp_decomp returns it), and for every row node r of level
  // L its final skeleton values S[r] (h x k, column-major) and global columns cols[r].  The
  // statistics, m_max_words included, come out as the depth-first construction would give
  // them for the same IDs.  The inputs are moved from.
  void assemble(std::vector<std::vector<IdResult>>& ids, std::vector<std::vector<double>>& S,
                std::vector<std::vector<int>>& cols);

  int rows() const { return rows_; }
  int cols() const { return cols_; }
  int C() const { return C_; }
  int L() const { return L_; }
  int ncol(int t) const { return 1 << (L_ - t); }
  int nrow(int t) const { return 1 << t; }
  int leaf_width(int c) const;
  int row_lo(int t, int r) const { return row_lo_[t][r]; }
  int row_hi(int t, int r) const { return row_lo_[t][r] + row_h_[t][r]; }
  int row_h(int t, int r) const { return row_h_[t][r]; }
  const BfBlock& block(int t, int r, int c) const { return blocks_[t][r * ncol(t) + c]; }
  const BfFinal& final_block(int r) const { return finals_[r]; }

  // rank statistics over every non-empty block (leaves and merges; a padded tree also has
  // empty slots, which k_max ignores by construction and n_ids / sum_k skip)
  // Serialised form of a complete tree (one record of the plan cache): shape, statistics,
  // every block and final skeleton.  load() rebuilds a tree that packs to the same factors;
  // it returns false (leaving the tree unusable) for a malformed or mismatched record.
  void save(std::vector<unsigned char>& out) const;
  bool load(const unsigned char* p, size_t n, int rows, int cols, int C, int L, double eps);

  int k_max = 0;
  long long n_ids = 0;
  double sum_k = 0.0, sum_k2 = 0.0;
  long long factor_entries = 0;  // T entries + final S entries
  long long words_now = 0, m_max_words = 0;
  double max_abs_t = 0.0;

 private:
  struct Pending {
    std::vector<double> vals;  // h x k column-major (skeleton columns on the block's rows)
    std::vector<int> gcols;
    bool live = false;
  };
  void merge(int t, int cc);
  void id_into(const double* a, int h, int K, int lda, BfBlock& blk, Pending& pend,
               const int* gcols);
  // Stores an ID as block blk and counts it in the statistics (h: the block's rows); take:
  // move the lists and T out of id instead of copying them.
  void record(IdResult& id, int h, int K, BfBlock& blk, bool take = false);

  int rows_ = 0, cols_ = 0, C_ = 1, L_ = 0;
  double eps_ = 0.0;
  int next_leaf_ = 0;
  std::vector<std::vector<int>> row_lo_, row_h_;
  std::vector<std::vector<BfBlock>> blocks_;
  std::vector<std::vector<Pending>> pending_;
  std::vector<BfFinal> finals_;
  IdWork work_;
  IdResult id_;
  std::vector<double> scratch_;
};

int butterfly_depth(int cols, int C);

// The n x n matrix of (transform) / (transform2) for order m and parity p (gauss_jacobi.cpp),
// column-major with leading dimension lda; threads = false computes it on the calling thread.
int gj_matrix(int m, int n, int p, double* a, int lda, bool threads);

}  // namespace sht
