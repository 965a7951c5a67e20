// Gauss-Legendre rule for the theta grid: the 2l zeros of P_{2l}, ascending
// (Section 2, equation (thetas)), with their weights.  Host FP64.
#include <algorithm>
#include <cmath>
#include <vector>

namespace sht {

// Evaluates P_n and P_{n-1} at x by the three-term recurrence in degree.
static inline void legendre_pair(int n, double x, double& pn, double& pn1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    pn = 1.0;
    pn1 = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pn1 = p0;
}

// Nodes ascending in x (x[i] = -x[n-1-i]) and weights w = 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  const int half = (n + 1) / 2;
  for (int i = 0; i < half; ++i) {
    // i-th largest zero: Tricomi-style first guess, then Newton.
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double pn = 0.0, pn1 = 0.0, dp = 1.0;
    int extra = 1;  // one more step after the correction drops below 1e-15
    for (int it = 0; it < 100; ++it) {
      legendre_pair(n, z, pn, pn1);
      dp = n * (z * pn - pn1) / ((z - 1.0) * (z + 1.0));
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-15 && it > 1 && extra-- == 0) break;
    }
    legendre_pair(n, z, pn, pn1);
    dp = n * (z * pn - pn1) / ((z - 1.0) * (z + 1.0));
    const double wi = 2.0 / ((1.0 - z) * (1.0 + z) * dp * dp);
    // z is the (i)-th largest: position n-1-i ascending; its mirror is -z at i.
    x[n - 1 - i] = z;
    w[n - 1 - i] = wi;
    x[i] = -z;
    w[i] = wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

}  // namespace sht
