// The per-order transforms of Section 4 on their own quadratures (host only): for order m,
// size n and parity p, the nodes are the n positive zeros of Pbar^m_{m+p+2n} (Lemma
// distinct_theorem: x_j for p = 0, y_j for p = 1), the weights those of Lemma quadratures,
// and the n x n matrix of (transform) / (transform2) is
//
//     A[i][j] = sqrt(w_i) Pbar^m_{m+p+2j}(x_i),   w = rho (p = 0) or sigma (p = 1),
//
// which is orthogonal.  Everything follows from the step-two recurrence (recurrence0),
// (recurrence) with the coefficients (c_rec), (d_rec): writing t = x^2 and
// Pbar^m_{m+p+2j}(x) = Pbar^m_{m+p}(x) Q_j(t), the polynomials Q_j satisfy
//
//     t Q_j = d_{l_j} Q_j + c_{l_j} Q_{j+1} + c_{l_{j-1}} Q_{j-1},   l_j = m + p + 2j,
//
// so the squared nodes are the eigenvalues of the symmetric tridiagonal matrix with
// diagonal d_{l_j} and off-diagonal c_{l_j} (j < n): they are found by Sturm-count
// bisection and polished by Newton's method on Q_n.  Because the rows of A have unit norm,
//
//     A[i][j] = Q_j(t_i) / ||Q(t_i)||,   1 / rho_i = Pbar^m_{m+p}(x_i)^2 ||Q(t_i)||^2,
//
// and the factor Pbar^m_{m+p}(x)^2 = C_m (1 - t)^m (times (2m + 3) t for p = 1), with
// C_m = (2m + 1)/2 prod_{k<=m} (2k - 1)/(2k) from (association), cancels from A.  The weights
// returned are lambda_i = w_i (1 - x_i^2)^m, those of the rule for the weight (1 - x^2)^m in
// Lemma quadratures, which stay within floating-point range for every m (rho alone carries
// (1 - x^2)^{-m}).  The paper finds its nodes by integrating an ODE in extended precision
// (Section 4, after its predecessor's Section 3.3); the eigenvalue route here is a
// different, standard method.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "interp_decomp.h"
#include "sht.h"

namespace {

double c_coef(double l, double m) {
  return std::sqrt((l - m + 1.0) * (l - m + 2.0) * (l + m + 1.0) * (l + m + 2.0) /
                   ((2.0 * l + 1.0) * (2.0 * l + 3.0) * (2.0 * l + 3.0) * (2.0 * l + 5.0)));
}
double d_coef(double l, double m) {
  return (2.0 * l * (l + 1.0) - 2.0 * m * m - 1.0) / ((2.0 * l - 1.0) * (2.0 * l + 3.0));
}

struct Jacobi {
  std::vector<double> a, b;  // diagonal (n), off-diagonal (n: b[n-1] links Q_{n-1} to Q_n)
  Jacobi(int m, int n, int p) : a(n), b(n) {
    for (int j = 0; j < n; ++j) {
      const double l = m + p + 2.0 * j;
      a[j] = d_coef(l, m);
      b[j] = c_coef(l, m);
    }
  }
  // Number of eigenvalues of the leading n x n block that are < t (Sturm sequence).
  int count_below(double t) const {
    const int n = static_cast<int>(a.size());
    int cnt = 0;
    double q = 1.0;
    for (int j = 0; j < n; ++j) {
      const double off = j ? b[j - 1] * b[j - 1] : 0.0;
      q = (a[j] - t) - (j ? off / q : 0.0);
      if (q == 0.0) q = -1e-300;  // t hit an eigenvalue of a leading block: nudge
      if (q < 0.0) ++cnt;
    }
    return cnt;
  }
  // Q_n(t) / Q_n'(t), from the recurrence and its derivative (rescaled jointly).
  double newton_ratio(double t) const {
    const int n = static_cast<int>(a.size());
    double q0 = 0.0, q1 = 1.0, d0 = 0.0, d1 = 0.0;  // Q_{j-1}, Q_j and their derivatives
    for (int j = 0; j < n; ++j) {
      const double bm = j ? b[j - 1] : 0.0;
      const double q2 = ((t - a[j]) * q1 - bm * q0) / b[j];
      const double d2 = (q1 + (t - a[j]) * d1 - bm * d0) / b[j];
      q0 = q1;
      q1 = q2;
      d0 = d1;
      d1 = d2;
      const double s = std::max(std::fabs(q1), std::fabs(d1));
      if (s > 1e150) {
        q0 /= s;
        q1 /= s;
        d0 /= s;
        d1 /= s;
      }
    }
    return q1 / d1;
  }
};

// Squared nodes t_0 < ... < t_{n-1} in (0, 1).
std::vector<double> squared_nodes(const Jacobi& J, int n) {
  std::vector<double> t(n);
  auto solve = [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      // Bisection isolates the i-th eigenvalue to a bracket of width 2^-40; the Sturm count
      // is exact only up to ~1e-16 absolute, which matters for the smallest t, so Newton on
      // Q_n finishes from there (it stays well inside the isolating bracket).
      double lo = 0.0, hi = 1.0;  // the zeros lie in (0, 1)
      for (int it = 0; it < 40; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (J.count_below(mid) > i)
          hi = mid;
        else
          lo = mid;
      }
      const double width = hi - lo;
      double x = 0.5 * (lo + hi);
      for (int it = 0; it < 8; ++it) {
        const double nx = x - J.newton_ratio(x);
        if (!(nx > lo - width && nx < hi + width)) break;
        const bool done = std::fabs(nx - x) <= 2e-16 * std::fabs(nx);
        x = nx;
        if (done) break;
      }
      t[i] = x;
    }
  };
  const int hw = sht::host_thread_count();
  const int nt = std::min(hw, std::max(1, n / 64));
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k) th.emplace_back(solve, static_cast<int>(static_cast<long long>(n) * k / nt),
                                                 static_cast<int>(static_cast<long long>(n) * (k + 1) / nt));
  for (auto& h : th) h.join();
  return t;
}

// Q_0 .. Q_{n-1} at t, all divided by one common factor, returned with the squared norm of
// that scaled vector; the rescaling keeps every entry finite.
double q_row(const Jacobi& J, int n, double t, double* q) {
  double qm = 0.0, qc = 1.0;
  q[0] = 1.0;
  for (int j = 0; j + 1 < n; ++j) {
    const double bm = j ? J.b[j - 1] : 0.0;
    const double qn = ((t - J.a[j]) * qc - bm * qm) / J.b[j];
    qm = qc;
    qc = qn;
    q[j + 1] = qc;
    const double s = std::fabs(qc);
    if (s > 1e150) {  // rescale the whole prefix and the running pair
      for (int k = 0; k <= j + 1; ++k) q[k] /= s;
      qm /= s;
      qc /= s;
    }
  }
  double ss = 0.0;
  for (int j = 0; j < n; ++j) ss += q[j] * q[j];
  return ss;
}

// log C_m with C_m = (2m + 1)/2 prod_{k=1..m} (2k - 1)/(2k).
double log_cm(int m) {
  double s = std::log((2.0 * m + 1.0) / 2.0);
  for (int k = 1; k <= m; ++k) s += std::log((2.0 * k - 1.0) / (2.0 * k));
  return s;
}

bool bad_args(int m, int n, int parity) {
  return m < 0 || n < 1 || (parity != 0 && parity != 1) || n > (1 << 24);
}

}  // namespace

extern "C" {

int sht_gj_rule(int m, int n, int parity, double* x, double* w) {
  if (bad_args(m, n, parity) || !x || !w) return SHT_EINVAL;
  const Jacobi J(m, n, parity);
  const std::vector<double> t = squared_nodes(J, n);
  const double lc = log_cm(m);
  for (int i = 0; i < n; ++i) {
    // lambda = 1 / (C_m ||Q||^2 [(2m + 3) t]), with ||Q||^2 = ss exp(2 log_scale) accumulated
    // alongside the rescaled recurrence.
    double qm = 0.0, qc = 1.0, log_scale = 0.0, ss = 1.0;
    for (int j = 0; j + 1 < n; ++j) {
      const double bm = j ? J.b[j - 1] : 0.0;
      const double qn = ((t[i] - J.a[j]) * qc - bm * qm) / J.b[j];
      qm = qc;
      qc = qn;
      ss += qc * qc;
      const double s = std::fabs(qc);
      if (s > 1e100) {
        qm /= s;
        qc /= s;
        ss /= s * s;
        log_scale += std::log(s);
      }
    }
    double lw = -lc - std::log(ss) - 2.0 * log_scale;
    if (parity == 1) lw -= std::log((2.0 * m + 3.0) * t[i]);
    x[i] = std::sqrt(t[i]);
    w[i] = std::exp(lw);
  }
  return SHT_OK;
}

int sht_gj_matrix(int m, int n, int parity, double* a, int lda) {
  if (bad_args(m, n, parity) || !a || lda < n) return SHT_EINVAL;
  const Jacobi J(m, n, parity);
  const std::vector<double> t = squared_nodes(J, n);
  auto rows = [&](int i0, int i1) {
    std::vector<double> q(n);
    for (int i = i0; i < i1; ++i) {
      const double inv = 1.0 / std::sqrt(q_row(J, n, t[i], q.data()));
      for (int j = 0; j < n; ++j) a[i + static_cast<long long>(j) * lda] = q[j] * inv;
    }
  };
  const int hw = sht::host_thread_count();
  const int nt = std::min(hw, std::max(1, n / 64));
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k) th.emplace_back(rows, static_cast<int>(static_cast<long long>(n) * k / nt),
                                                 static_cast<int>(static_cast<long long>(n) * (k + 1) / nt));
  for (auto& h : th) h.join();
  return SHT_OK;
}

}  // extern "C"
