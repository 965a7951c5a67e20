// Legendre column generator (FP64, GPU).
//
// Column j of Q^{(m,p)} holds sqrt(2 w_i) Pbar^m_{m+p+2j}(x_i) on the l positive
// Gauss-Legendre nodes.  One thread owns one (pair, node) and walks the degree
// with the step-two recurrence of Lemma rec_relation,
//   x^2 P_d = c_{d-2} P_{d-2} + d_d P_d + c_d P_{d+2}     (recurrence)
//   x^2 P_d = d_d P_d + c_d P_{d+2},  d = m, m+1          (recurrence0)
// with c_d, d_d from (c_rec), (d_rec), seeded by Pbar_m^m and Pbar_{m+1}^m from
// (association).  Values are carried as mantissa * 2^e (explicit exponent
// tracking, Section 5) so that seeds far below the FP64 range still grow into
// the band where the functions are O(1).
//
// On the common Gauss-Legendre grid the recurrence meets nodes next to the
// equator (x ~ 0) and the poles (x ~ 1), where its characteristic roots
// coalesce (r ~ -1 and r ~ +1) and rounding errors grow linearly with the
// degree.  The state and the coefficients are therefore carried as unevaluated
// sums of two doubles (double-double), which keeps the columns accurate to the
// final FP64 rounding; the output is plain FP64.
//
// The recurrence state survives between launches, so the columns are produced
// leaf chunk by leaf chunk in the order the depth-first precompute consumes
// them (Section 4).
#include "sht_internal.h"

#pragma clang fp contract(off)

namespace sht {

namespace {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  const double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e = fma(a.hi, b.lo, e);
  e = fma(a.lo, b.hi, e);
  return quick_two_sum(p, e);
}

__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  const double p = a.hi * b;
  double e = fma(a.hi, b, -p);
  e = fma(a.lo, b, e);
  return quick_two_sum(p, e);
}

__device__ __forceinline__ dd dd_div(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_neg(dd_mul_d(b, q1)));
  const double q2 = r.hi / b.hi;
  r = dd_add(r, dd_neg(dd_mul_d(b, q2)));
  const double q3 = r.hi / b.hi;
  return dd_add(quick_two_sum(q1, q2), dd{q3, 0.0});
}

__device__ __forceinline__ dd dd_sqrt(dd a) {
  if (a.hi <= 0.0) return {0.0, 0.0};
  const double x = sqrt(a.hi);
  const double p = x * x;
  const double e = fma(x, x, -p);
  const double corr = (((a.hi - p) - e) + a.lo) / (2.0 * x);
  return quick_two_sum(x, corr);
}

__device__ __forceinline__ dd dd_ratio(double num, double den) { return dd_div(dd{num, 0.0}, dd{den, 0.0}); }

// (c_rec): c_d = sqrt((d-m+1)(d-m+2)(d+m+1)(d+m+2) / ((2d+1)(2d+3)^2(2d+5))); both
// products are integers below 2^53 for degrees < 8192, hence exact in FP64.
__device__ __forceinline__ dd c_rec(double d, double m) {
  const double num = (d - m + 1.0) * (d - m + 2.0) * (d + m + 1.0) * (d + m + 2.0);
  const double den = (2.0 * d + 1.0) * (2.0 * d + 3.0) * (2.0 * d + 3.0) * (2.0 * d + 5.0);
  return dd_sqrt(dd_ratio(num, den));
}

// (d_rec): d_d = (2d(d+1) - 2m^2 - 1) / ((2d-1)(2d+3)).
__device__ __forceinline__ dd d_rec(double d, double m) {
  return dd_ratio(2.0 * d * (d + 1.0) - 2.0 * m * m - 1.0, (2.0 * d - 1.0) * (2.0 * d + 3.0));
}

__device__ __forceinline__ dd dd_scale(dd a, double s) { return {a.hi * s, a.lo * s}; }

}  // namespace

__global__ void k_legendre_seed(int npairs, int l, const int* __restrict__ mm,
                                const int* __restrict__ pp, const double* __restrict__ x,
                                double2* __restrict__ prev, double2* __restrict__ cur,
                                int* __restrict__ ex) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= npairs || i >= l) return;
  const int m = mm[b], p = pp[b];
  const double xi = x[i];
  const dd x2{xi * xi, fma(xi, xi, -(xi * xi))};
  const dd s = dd_sqrt(dd_add(dd{1.0, 0.0}, dd_neg(quick_two_sum(x2.hi, x2.lo))));
  // Pbar_m^m = sqrt((2m+1)/2 * prod_{j<=m} (2j-1)/(2j)) (1 - x^2)^{m/2}   (association)
  dd mant = dd_sqrt(dd_ratio(2.0 * m + 1.0, 2.0));
  int e = 0;
  for (int j = 1; j <= m; ++j) {
    mant = dd_mul(dd_mul(mant, dd_sqrt(dd_ratio(2.0 * j - 1.0, 2.0 * j))), s);
    if (fabs(mant.hi) < 0x1p-400) {
      mant = dd_scale(mant, 0x1p400);
      e -= 400;
    }
  }
  dd c = mant;
  if (p == 1) c = dd_mul_d(dd_mul(dd_sqrt(dd{2.0 * m + 3.0, 0.0}), mant), xi);  // Pbar_{m+1}^m
  const size_t o = static_cast<size_t>(b) * l + i;
  prev[o] = make_double2(0.0, 0.0);
  cur[o] = make_double2(c.hi, c.lo);
  ex[o] = e;
}

__global__ void k_legendre_chunk(int npairs, int l, int C, int chunk, const int* __restrict__ mm,
                                 const int* __restrict__ pp, const int* __restrict__ nc,
                                 const double* __restrict__ x, const double* __restrict__ sw,
                                 double2* __restrict__ prev, double2* __restrict__ cur,
                                 int* __restrict__ ex, double* __restrict__ out) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= npairs || i >= l) return;
  const int m = mm[b], p = pp[b], n = nc[b];
  const int j0 = chunk * C;
  const int width = min(C, n - j0);
  if (width <= 0) return;
  const size_t o = static_cast<size_t>(b) * l + i;
  const double xi = x[i];
  const dd x2{xi * xi, fma(xi, xi, -(xi * xi))};
  const double swi = sw[i];
  const double md = static_cast<double>(m);
  dd P0{prev[o].x, prev[o].y};
  dd P1{cur[o].x, cur[o].y};
  int e = ex[o];
  double* dst = out + static_cast<size_t>(b) * C * l + i;
  for (int jj = 0; jj < width; ++jj) {
    const int j = j0 + jj;
    if (j > 0) {
      const double d = static_cast<double>(m + p + 2 * (j - 1));  // degree of P1
      dd num = dd_mul(dd_add(x2, dd_neg(d_rec(d, md))), P1);
      if (d >= md + 2.0) num = dd_add(num, dd_neg(dd_mul(c_rec(d - 2.0, md), P0)));
      const dd P2 = dd_div(num, c_rec(d, md));
      P0 = P1;
      P1 = P2;
      if (fabs(P1.hi) > 0x1p400) {
        P1 = dd_scale(P1, 0x1p-400);
        P0 = dd_scale(P0, 0x1p-400);
        e += 400;
      }
    }
    dst[static_cast<size_t>(jj) * l] = ldexp(P1.hi + P1.lo, e) * swi;
  }
  prev[o] = make_double2(P0.hi, P0.lo);
  cur[o] = make_double2(P1.hi, P1.lo);
  ex[o] = e;
}

hipError_t legendre_seed(ColumnBatch& b, hipStream_t s) {
  dim3 grid((b.l + 255) / 256, b.npairs);
  hipLaunchKernelGGL(k_legendre_seed, grid, dim3(256), 0, s, b.npairs, b.l, b.d_m, b.d_p, b.d_x,
                     reinterpret_cast<double2*>(b.d_prev), reinterpret_cast<double2*>(b.d_cur),
                     b.d_exp);
  return hipGetLastError();
}

hipError_t legendre_chunk(ColumnBatch& b, int chunk, hipStream_t s) {
  dim3 grid((b.l + 255) / 256, b.npairs);
  hipLaunchKernelGGL(k_legendre_chunk, grid, dim3(256), 0, s, b.npairs, b.l, b.C, chunk, b.d_m,
                     b.d_p, b.d_ncols, b.d_x, b.d_sw, reinterpret_cast<double2*>(b.d_prev),
                     reinterpret_cast<double2*>(b.d_cur), b.d_exp, b.d_out);
  return hipGetLastError();
}

}  // namespace sht
