// The per-order transforms of Section 5 on their own quadratures (host only): for order m,
// size n and parity p, the nodes are the n positive zeros of Pbar^m_L, L = m + p + 2n (Lemma
// distinct_theorem: x_j for p = 0, y_j for p = 1), the weights those of Lemma quadratures,
// and the n x n matrix of (transform) / (transform2) is
//
//     A[i][j] = sqrt(w_i) Pbar^m_{m+p+2j}(x_i),   w = rho (p = 0) or sigma (p = 1),
//
// which is orthogonal.
//
// Isolation.  With t = x^2 and Pbar^m_{m+p+2j}(x) = Pbar^m_{m+p}(x) Q_j(t), the step-two
// recurrence (recurrence0), (recurrence) with the coefficients (c_rec), (d_rec) reads
//
//     t Q_j = d_{l_j} Q_j + c_{l_j} Q_{j+1} + c_{l_{j-1}} Q_{j-1},   l_j = m + p + 2j,
//
// so the squared nodes are the eigenvalues of the symmetric tridiagonal matrix with diagonal
// d_{l_j} and off-diagonal c_{l_j}: Sturm-count bisection isolates each one.
//
// Refinement and evaluation.  Near the equator t is tiny and t - d_{l_j} keeps only its
// leading bits, so the nodes are finished, and the weights and matrix rows evaluated, in x
// with the normalized three-term recurrence of the functions themselves: writing
// Pbar^m_d(x) = Pbar^m_m(x) R_d(x),
//
//     R_m = 1,  R_{m+1} = sqrt(2m + 3) x,  a_{d+1} R_{d+1} = x R_d - a_d R_{d-1},
//     a_d = sqrt((d^2 - m^2) / (4 d^2 - 1)),
//
// which involves x only through products.  Newton's method on R_L gives the nodes.  Since
// Pbar^m_m(x)^2 = C_m (1 - x^2)^m with C_m = (2m + 1)/2 prod_{k<=m} (2k - 1)/(2k) from
// (association), the weights of (weights1) / (weights2) become
//
//     lambda_i = w_i (1 - x_i^2)^m = 2 (2L + 1) / ((1 - x_i^2) C_m R_L'(x_i)^2),
//
// the weights of the rule for (1 - x^2)^m in Lemma quadratures, which stay in range for every
// m (w alone carries (1 - x^2)^-m).  The rows of A have unit norm, so A[i][j] =
// R_{m+p+2j}(x_i) / ||(R_{m+p+2k}(x_i))_k||, where the seed factor cancels.  The paper finds
// its nodes by integrating an ODE in extended precision (Section 5, after its predecessor's
// Section 3.3); this is a different, standard route.
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

// The tridiagonal matrix of the step-two recurrence in t, for the Sturm counts.
struct Jacobi {
  std::vector<double> a, b2;  // diagonal (n), squared off-diagonal (n - 1)
  Jacobi(int m, int n, int p) : a(n), b2(n > 1 ? n - 1 : 0) {
    for (int j = 0; j < n; ++j) {
      const double l = m + p + 2.0 * j;
      a[j] = d_coef(l, m);
      if (j + 1 < n) {
        const double c = c_coef(l, m);
        b2[j] = c * c;
      }
    }
  }
  // Number of eigenvalues below t.
  int count_below(double t) const {
    const int n = static_cast<int>(a.size());
    int cnt = 0;
    double q = 1.0;
    for (int j = 0; j < n; ++j) {
      q = (a[j] - t) - (j ? b2[j - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;  // t hit an eigenvalue of a leading block: nudge
      if (q < 0.0) ++cnt;
    }
    return cnt;
  }
};

// The normalized recurrence in x for degrees m .. L.
struct StepOne {
  int m, L;
  std::vector<double> a;  // a[d - m] = a_d for d = m + 1 .. L + 1 (a[0] unused)
  StepOne(int m_, int L_) : m(m_), L(L_), a(L_ - m_ + 2, 0.0) {
    for (int d = m + 1; d <= L + 1; ++d)
      a[d - m] = std::sqrt((static_cast<double>(d) - m) * (static_cast<double>(d) + m) /
                           ((2.0 * d - 1.0) * (2.0 * d + 1.0)));
  }
  // R_L(x) / R_L'(x), and log |R_L'(x)|; value and derivative are rescaled together.
  void newton(double x, double& ratio, double& log_deriv) const {
    double r0 = 1.0, r1 = std::sqrt(2.0 * m + 3.0) * x;
    double d0 = 0.0, d1 = std::sqrt(2.0 * m + 3.0);
    double log_scale = 0.0;
    for (int d = m + 1; d < L; ++d) {
      const double an = a[d + 1 - m], ad = a[d - m];
      const double r2 = (x * r1 - ad * r0) / an;
      const double d2 = (r1 + x * d1 - ad * d0) / an;
      r0 = r1;
      r1 = r2;
      d0 = d1;
      d1 = d2;
      const double s = std::max(std::fabs(r1), std::fabs(d1));
      if (s > 1e150) {
        r0 /= s;
        r1 /= s;
        d0 /= s;
        d1 /= s;
        log_scale += std::log(s);
      }
    }
    ratio = r1 / d1;
    log_deriv = std::log(std::fabs(d1)) + log_scale;
  }
  // R_{m+p+2j}(x) for j < n into q, all divided by one common factor (rescaled so every
  // entry stays finite); returns the squared norm of the scaled vector.
  double row(double x, int p, int n, double* q) const {
    double r0 = 1.0, r1 = std::sqrt(2.0 * m + 3.0) * x;
    int filled = 0;
    q[filled++] = p == 0 ? r0 : r1;
    for (int d = m + 1; filled < n; ++d) {
      const double r2 = (x * r1 - a[d - m] * r0) / a[d + 1 - m];
      r0 = r1;
      r1 = r2;
      if (((d + 1 - m - p) & 1) == 0) q[filled++] = r1;  // degree d + 1 = m + p + 2j
      const double s = std::max(std::fabs(r0), std::fabs(r1));
      if (s > 1e150) {  // rescale the stored prefix and the running pair
        for (int k = 0; k < filled; ++k) q[k] /= s;
        r0 /= s;
        r1 /= s;
      }
    }
    double ss = 0.0;
    for (int j = 0; j < n; ++j) ss += q[j] * q[j];
    return ss;
  }
};

// log C_m with C_m = (2m + 1)/2 prod_{k=1..m} (2k - 1)/(2k).
double log_cm(int m) {
  double s = std::log((2.0 * m + 1.0) / 2.0);
  for (int k = 1; k <= m; ++k) s += std::log((2.0 * k - 1.0) / (2.0 * k));
  return s;
}

bool bad_args(int m, int n, int parity) {
  return m < 0 || n < 1 || (parity != 0 && parity != 1) || n > (1 << 24);
}

template <typename F>
void split_range(int n, F&& fn, bool threads = true) {
  const int nt = threads ? std::min(sht::host_thread_count(), std::max(1, n / 64)) : 1;
  if (nt == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k)
    th.emplace_back(fn, static_cast<int>(static_cast<long long>(n) * k / nt),
                    static_cast<int>(static_cast<long long>(n) * (k + 1) / nt));
  for (auto& h : th) h.join();
}

// Nodes x_0 < ... < x_{n-1} in (0, 1), with log |R_L'| at each.
void nodes(int m, int n, int p, std::vector<double>& x, std::vector<double>& log_deriv, bool threads = true) {
  const Jacobi J(m, n, p);
  const StepOne S(m, m + p + 2 * n);
  x.assign(n, 0.0);
  log_deriv.assign(n, 0.0);
  split_range(n, [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      // bisection on t to a bracket of width 2^-44 (the Sturm count is exact to ~1e-16 in t,
      // far below the spacing of the squared nodes)
      double lo = 0.0, hi = 1.0;
      for (int it = 0; it < 44; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (J.count_below(mid) > i)
          hi = mid;
        else
          lo = mid;
      }
      const double xlo = std::sqrt(lo), xhi = std::sqrt(hi), w = xhi - xlo;
      double xi = 0.5 * (xlo + xhi), ratio = 0.0, ld = 0.0;
      for (int it = 0; it < 12; ++it) {
        S.newton(xi, ratio, ld);
        const double nx = xi - ratio;
        if (!(nx > xlo - w && nx < xhi + w)) break;  // stay in the isolating bracket
        const bool done = std::fabs(nx - xi) <= 1e-16 * nx;
        xi = nx;
        if (done) break;
      }
      S.newton(xi, ratio, ld);
      x[i] = xi;
      log_deriv[i] = ld;
    }
  }, threads);
}

}  // namespace

namespace sht {

int gj_matrix(int m, int n, int parity, double* a, int lda, bool threads) {
  if (bad_args(m, n, parity) || !a || lda < n) return SHT_EINVAL;
  std::vector<double> xs, ld;
  nodes(m, n, parity, xs, ld, threads);
  const StepOne S(m, m + parity + 2 * n);
  split_range(n, [&](int i0, int i1) {
    std::vector<double> q(n);
    for (int i = i0; i < i1; ++i) {
      const double inv = 1.0 / std::sqrt(S.row(xs[i], parity, n, q.data()));
      for (int j = 0; j < n; ++j) a[i + static_cast<long long>(j) * lda] = q[j] * inv;
    }
  }, threads);
  return SHT_OK;
}

}  // namespace sht

extern "C" {

int sht_gj_rule(int m, int n, int parity, double* x, double* w) {
  if (bad_args(m, n, parity) || !x || !w) return SHT_EINVAL;
  std::vector<double> xs, ld;
  nodes(m, n, parity, xs, ld);
  const double L = m + parity + 2.0 * n;
  const double lc = log_cm(m);
  for (int i = 0; i < n; ++i) {
    x[i] = xs[i];
    // 1 - x^2 as (1 - x)(1 + x): 1 - x is exact near the pole, where x * x would round
    w[i] = std::exp(std::log(2.0 * (2.0 * L + 1.0)) - std::log1p(-xs[i]) - std::log1p(xs[i]) - lc -
                    2.0 * ld[i]);
  }
  return SHT_OK;
}

int sht_gj_matrix(int m, int n, int parity, double* a, int lda) {
  return sht::gj_matrix(m, n, parity, a, lda, true);
}

}  // extern "C"
