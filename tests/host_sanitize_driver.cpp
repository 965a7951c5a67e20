// Drives the host-only parts of the library (interpolative decompositions and depth-first
// butterflies of random matrices of many shapes, leaf widths and ranks; the per-order rules
// and matrices; the Gauss-Legendre rule) in a build with address and undefined-behaviour
// sanitizers.  Built and run by tests/test_host_library.py; prints "drv ok".
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "interp_decomp.h"
#include "sht.h"
namespace sht { void gauss_legendre(int n, double* x, double* w); }
int main() {
  std::mt19937_64 g(5);
  std::normal_distribution<double> N(0, 1);
  // butterflies of random low-rank-ish matrices, several shapes, leaf widths and depths
  for (int trial = 0; trial < 200; ++trial) {
    int rows = 1 + g() % 90, cols = g() % 90, C = 1 + g() % 17;
    int L = sht::butterfly_depth(cols, C);
    if ((1 << L) > rows) continue;
    int r = 1 + g() % 12;
    std::vector<double> U(rows * r), V(r * std::max(cols, 1)), A(rows * std::max(cols, 1));
    for (auto& v : U) v = N(g);
    for (auto& v : V) v = N(g);
    for (int j = 0; j < cols; ++j)
      for (int i = 0; i < rows; ++i) {
        double s = 0; for (int q = 0; q < r; ++q) s += U[i + q * rows] * V[q + j * r];
        A[i + j * rows] = s * std::exp(0.3 * N(g)) + 1e-9 * N(g);
      }
    sht::BfTree t;
    const double eps = std::pow(10.0, -3.0 - (g() % 11));
    t.init(rows, cols, C, L, eps);
    for (int c = 0; c < (1 << L); ++c) {
      const double* chunk = A.data() + (size_t)c * C * rows;
      if (t.leaf_width(c) == 0) chunk = A.data();
      t.add_leaf(c, chunk, rows);
    }
    // the same tree assembled from its own IDs and finals (the device builder's path) must
    // serialise to the same bytes, statistics and depth-first memory figure included
    std::vector<std::vector<sht::IdResult>> ids(L + 1);
    for (int lv = 0; lv <= L; ++lv)
      for (int rr = 0; rr < t.nrow(lv); ++rr)
        for (int cc = 0; cc < t.ncol(lv); ++cc) {
          const sht::BfBlock& b = t.block(lv, rr, cc);
          sht::IdResult id;
          id.k = b.k;
          id.skel = b.skel;
          id.red = b.red;
          id.T = b.T;
          for (double v : b.T) id.max_abs_t = std::max(id.max_abs_t, std::fabs(v));
          ids[lv].push_back(id);
        }
    std::vector<std::vector<double>> S;
    std::vector<std::vector<int>> fc;
    for (int rr = 0; rr < (1 << L); ++rr) {
      S.push_back(t.final_block(rr).S);
      fc.push_back(t.final_block(rr).cols);
    }
    sht::BfTree t2;
    t2.init(rows, cols, C, L, eps);
    t2.assemble(ids, S, fc);
    std::vector<unsigned char> a1, a2;
    t.save(a1);
    t2.save(a2);
    if (a1 != a2 || !t2.complete()) {
      std::printf("assemble mismatch in trial %d\n", trial);
      return 3;
    }
  }
  // per-order rules and matrices
  int cases[][3] = {{0,1,0},{0,1,1},{3,7,0},{500,2,1},{40,33,1},{0,130,0},{200,200,1}};
  for (auto& cs : cases) {
    int m = cs[0], n = cs[1], p = cs[2];
    std::vector<double> x(n), w(n), a((size_t)n * (n + 1));
    if (sht_gj_rule(m, n, p, x.data(), w.data()) != SHT_OK) return 1;
    if (sht_gj_matrix(m, n, p, a.data(), n + 1) != SHT_OK) return 2;
  }
  for (int n : {1, 2, 3, 17, 64, 255}) {
    std::vector<double> x(n), w(n);
    sht::gauss_legendre(n, x.data(), w.data());
  }
  std::puts("drv ok");
  return 0;
}
