/*
 * Oracle: table of normalized associated Legendre functions for one order, in plain C.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load this library; the GPU library shares no code with it.
 *
 * Same definition and the same step-one recurrence as oracle/legendre.py (which the tests
 * pin this file against, beside the pins of the functions themselves), written as plain
 * loops per node so that the oracle can cover every order of the largest bandlimits:
 *
 *   Pbar_m^m(x)     = sqrt((2m+1)/2 * prod_{j=1..m} (2j-1)/(2j)) (1 - x^2)^{m/2}
 *                     (Section 2.3, equation (association), no Condon-Shortley phase),
 *   Pbar_{m+1}^m(x) = sqrt(2m+3) x Pbar_m^m(x),
 *   x Pbar_k = a_{k+1} Pbar_{k+1} + a_k Pbar_{k-1},  a_k = sqrt((k^2 - m^2) / (4k^2 - 1)).
 *
 * This is the classical first-order-in-degree recurrence, deliberately not the step-two
 * recurrence (recurrence0) / (recurrence) of the GPU column kernel.  Underflow of the seed
 * at large m is handled by explicit exponent tracking (Section 4): each value is a mantissa
 * times 2^e with an integer e, rescaled by 2^400 whenever the mantissa leaves
 * [2^-400, 2^400]; values below the FP64 range are written as 0.
 */
#include <math.h>

#define BIG 0x1p400
#define SMALL 0x1p-400
#define STEP 400

/* out[(k - m) * n + i] = Pbar_k^m(x[i]) for k = m..kmax and i = 0..n-1.  The recurrence runs
 * degree by degree over all nodes; `work` holds 3 n doubles (previous value, current value,
 * exponent of each node).  Returns 0, or -1 for m < 0, kmax < m, n < 0 or a null pointer. */
int oracle_pbar_table(int m, int kmax, const double* x, int n, double* out, double* work) {
  if (m < 0 || kmax < m || n < 0 || !x || !out || !work) return -1;
  double* prev = work;
  double* cur = work + n;
  double* ex = work + 2 * (long)n; /* integer exponents, held exactly as doubles */
  /* seeds: running product of sqrt((2j-1)/(2j)) (1 - x^2)^{1/2}, with its exponent */
  for (int i = 0; i < n; ++i) {
    const double s = sqrt((1.0 - x[i]) * (1.0 + x[i]));
    double mant = 1.0, e = 0.0;
    for (int j = 1; j <= m; ++j) {
      mant *= sqrt((2.0 * j - 1.0) / (2.0 * j)) * s;
      if (mant != 0.0 && fabs(mant) < SMALL) {
        mant *= BIG;
        e -= STEP;
      }
    }
    prev[i] = 0.0;
    cur[i] = sqrt((2.0 * m + 1.0) / 2.0) * mant; /* Pbar_m^m */
    ex[i] = e;
    out[i] = ldexp(cur[i], (int)(e < -100000.0 ? -100000.0 : e));
  }
  const double mm = (double)m;
  for (int k = m; k < kmax; ++k) {
    /* Pbar_{k+1} = (x Pbar_k - a_k Pbar_{k-1}) / a_{k+1}; a_m = 0 */
    const double kk = (double)k, k1 = (double)(k + 1);
    const double a_k = k > m ? sqrt((kk * kk - mm * mm) / (4.0 * kk * kk - 1.0)) : 0.0;
    const double a_k1 = sqrt((k1 * k1 - mm * mm) / (4.0 * k1 * k1 - 1.0));
    double* row = out + (long)(k + 1 - m) * n;
    for (int i = 0; i < n; ++i) {
      double nxt = (x[i] * cur[i] - a_k * prev[i]) / a_k1;
      double c = cur[i];
      if (fabs(nxt) > BIG) {
        nxt *= SMALL;
        c *= SMALL;
        ex[i] += STEP;
      }
      prev[i] = c;
      cur[i] = nxt;
      if (ex[i] == 0.0) {
        row[i] = nxt;
      } else {
        const double e = ex[i] < -100000.0 ? -100000.0 : (ex[i] > 100000.0 ? 100000.0 : ex[i]);
        row[i] = ldexp(nxt, (int)e);
      }
    }
  }
  return 0;
}
