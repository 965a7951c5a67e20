// Butterfly apply kernels: synthesis direction (Q = S * T_L * ... * T_leaf) and the
// transposed direction that analysis and the adjoint need (Section 3.2 and the remark
// after equation (bottom): one factorization serves A and A^T).
//
// Data live in R-wide rows: R = 4F for complex fields (re/im of +m and -m per field),
// R = 2F for real fields.  A work-group takes one task and a tile of RT columns; the
// task's input rows are staged in LDS, the factor entries stream from HBM in the order
// the plan packed them (column-major T, so consecutive lanes read consecutive words).
#include <algorithm>

#include "sht_internal.h"

namespace sht {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ long long coeff_offset(int l, int m, int kind) {
  const long long L2 = 2LL * l;
  if (kind == SHT_REAL) return static_cast<long long>(m) * L2 - static_cast<long long>(m) * (m - 1) / 2;
  if (m == 0) return 0;
  return L2 + 2LL * (m - 1) * L2 - static_cast<long long>(m - 1) * m;
}

// ------------------------------------------------------------------------------- layout
// S1: canonical coefficients -> internal rows [pair][j][R]; zero where no entry exists.
__global__ void k_coeff_to_xin(const PairDesc* __restrict__ pairs, const double* __restrict__ coeff,
                               double* __restrict__ xin, int l, int F, int R, int kind,
                               long long ncoef) {
  const PairDesc pd = pairs[blockIdx.x];
  const int m = pd.m, p = pd.p, n = pd.n;
  const long long base = coeff_offset(l, m, kind);
  const int L2 = 2 * l;
  const long long total = static_cast<long long>(n) * R;
  for (long long e = blockIdx.y * kThreads + threadIdx.x; e < total; e += gridDim.y * kThreads) {
    const int j = static_cast<int>(e / R);
    const int col = static_cast<int>(e % R);
    const int k = m + p + 2 * j;
    double v = 0.0;
    if (kind == SHT_COMPLEX) {
      const int f = col >> 2, s = (col >> 1) & 1, c = col & 1;
      if (!(m == 0 && s == 1)) {
        const long long sidx = base + (s ? (L2 - m) : 0) + (k - m);
        v = coeff[(static_cast<long long>(f) * ncoef + sidx) * 2 + c];
      }
    } else {
      const int f = col >> 1, c = col & 1;
      if (!(m == 0 && c == 1)) v = coeff[(static_cast<long long>(f) * ncoef + base + (k - m)) * 2 + c];
    }
    xin[(static_cast<long long>(pd.in_base) + j) * R + col] = v;
  }
}

// N5: internal rows -> canonical coefficients.
__global__ void k_xin_to_coeff(const PairDesc* __restrict__ pairs, const double* __restrict__ xin,
                               double* __restrict__ coeff, int l, int F, int R, int kind,
                               long long ncoef) {
  const PairDesc pd = pairs[blockIdx.x];
  const int m = pd.m, p = pd.p, n = pd.n;
  const long long base = coeff_offset(l, m, kind);
  const int L2 = 2 * l;
  const long long total = static_cast<long long>(n) * R;
  for (long long e = blockIdx.y * kThreads + threadIdx.x; e < total; e += gridDim.y * kThreads) {
    const int j = static_cast<int>(e / R);
    const int col = static_cast<int>(e % R);
    const int k = m + p + 2 * j;
    const double v = xin[(static_cast<long long>(pd.in_base) + j) * R + col];
    if (kind == SHT_COMPLEX) {
      const int f = col >> 2, s = (col >> 1) & 1, c = col & 1;
      if (m == 0 && s == 1) continue;
      const long long sidx = base + (s ? (L2 - m) : 0) + (k - m);
      coeff[(static_cast<long long>(f) * ncoef + sidx) * 2 + c] = v;
    } else {
      const int f = col >> 1, c = col & 1;
      coeff[(static_cast<long long>(f) * ncoef + base + (k - m)) * 2 + c] = (m == 0 && c == 1) ? 0.0 : v;
    }
  }
}

// ------------------------------------------------------------------------------- levels
// Few columns per (m, p) (R below the matrix-core width): every factor word is used R times,
// so these launches stream the factors.  One thread owns one output row for all RT columns of
// the work-group's tile (RT accumulators), and walks the contraction with kUnroll factor
// loads in flight; consecutive lanes take consecutive rows, so a wave's factor loads are
// 512 contiguous bytes of a column-major T (synthesis) or of its transposed copy (transposed
// apply).  The vector operands sit in LDS and are read as broadcasts.
constexpr int kVecThreads = 128;  // two waves: typically one per output block of a task
constexpr int kUnroll = 8;

// Synthesis: out_o = in[skel_o] + T_o in[red_o] for the task's one or two outputs.  Tasks
// whose input rows are coefficients (mp >= 0: leaves) read them from the internal rows `xin`.
template <int RT>
__global__ void __launch_bounds__(kVecThreads)
k_level_synth(const LevelTask* __restrict__ tasks, const double* __restrict__ fac,
              const uint16_t* __restrict__ idx, const double* __restrict__ in,
              const double* __restrict__ xin, double* __restrict__ out, int R) {
  extern __shared__ double lds[];
  const LevelTask& tk = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const int K = tk.K;
  const int k0 = tk.k[0], k1 = tk.k[1] < 0 ? 0 : tk.k[1];
  const double* src = tk.mp >= 0 ? xin : in;
  double* x = lds;                                         // K x RT
  uint16_t* ix = reinterpret_cast<uint16_t*>(lds + K * RT);  // [skel0 red0 | skel1 red1]
  for (int e = threadIdx.x; e < K * RT; e += kVecThreads)
    x[e] = src[(static_cast<long long>(tk.in_row) + e / RT) * R + r0 + e % RT];
  for (int e = threadIdx.x; e < K; e += kVecThreads) {
    ix[e] = idx[tk.idx[0] + e];
    if (k1 > 0) ix[K + e] = idx[tk.idx[1] + e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nc0 = (k0 + 63) >> 6, nc1 = (k1 + 63) >> 6;
  for (int it = wave; it < nc0 + nc1; it += kVecThreads / 64) {
    const int o = it < nc0 ? 0 : 1;
    const int k = o ? k1 : k0;
    const int i = (o ? it - nc0 : it) * 64 + lane;
    if (i >= k) continue;
    const uint16_t* skel = ix + o * K;
    const uint16_t* red = skel + k;
    const int nr = K - k;
    const double* T = fac + tk.fac[o] + i;  // T (k x nr, column-major): entry (i, j) at j k + i
    double acc[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) acc[c] = 0.0;
    int j = 0;
    for (; j + kUnroll <= nr; j += kUnroll) {
      double t[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) t[u] = T[static_cast<long long>(j + u) * k];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const double* xr = x + red[j + u] * RT;
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[c] = fma(t[u], xr[c], acc[c]);
      }
    }
    for (; j < nr; ++j) {
      const double t = T[static_cast<long long>(j) * k];
      const double* xr = x + red[j] * RT;
#pragma unroll
      for (int c = 0; c < RT; ++c) acc[c] = fma(t, xr[c], acc[c]);
    }
    const double* xs = x + skel[i] * RT;
    double* dst = out + (static_cast<long long>(tk.out_row[o]) + i) * R + r0;
#pragma unroll
    for (int c = 0; c < RT; ++c) dst[c] = xs[c] + acc[c];
  }
}

// Transposed: in = sum_o (Ã_o)^T out_o, where Ã_o has the identity at skel_o and T_o at red_o.
// Each input row receives exactly one term from each output block (its identity row or its
// T^T row), added into a zeroed LDS block, so the result does not depend on the order.
template <int RT>
__global__ void __launch_bounds__(kVecThreads)
k_level_trans(const LevelTask* __restrict__ tasks, const double* __restrict__ fac,
              const uint16_t* __restrict__ idx, const double* __restrict__ win,
              double* __restrict__ xout, double* __restrict__ xin, int R) {
  extern __shared__ double lds[];
  const LevelTask& tk = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const int K = tk.K;
  const int k0 = tk.k[0];
  const int k1 = tk.k[1] < 0 ? 0 : tk.k[1];
  const int nouts = tk.k[1] < 0 ? 1 : 2;
  double* acc_l = lds;              // K x RT
  double* w0 = acc_l + K * RT;      // k0 x RT
  double* w1 = w0 + k0 * RT;        // k1 x RT
  uint16_t* ix = reinterpret_cast<uint16_t*>(w1 + k1 * RT);
  for (int e = threadIdx.x; e < K * RT; e += kVecThreads) acc_l[e] = 0.0;
  for (int e = threadIdx.x; e < k0 * RT; e += kVecThreads)
    w0[e] = win[(static_cast<long long>(tk.out_row[0]) + e / RT) * R + r0 + e % RT];
  for (int e = threadIdx.x; e < k1 * RT; e += kVecThreads)
    w1[e] = win[(static_cast<long long>(tk.out_row[1]) + e / RT) * R + r0 + e % RT];
  for (int e = threadIdx.x; e < K; e += kVecThreads) {
    ix[e] = idx[tk.idx[0] + e];
    if (nouts > 1) ix[K + e] = idx[tk.idx[1] + e];
  }
  __syncthreads();
  // identity rows
  for (int o = 0; o < nouts; ++o) {
    const int k = o ? k1 : k0;
    const double* w = o ? w1 : w0;
    const uint16_t* skel = ix + o * K;
    for (int e = threadIdx.x; e < k * RT; e += kVecThreads)
      atomicAdd(acc_l + skel[e / RT] * RT + e % RT, w[e]);
  }
  // T^T rows: one thread per redundant column j of an output, summed over that output's rows
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nr0 = K - k0, nr1 = nouts > 1 ? K - k1 : 0;
  const int nc0 = (nr0 + 63) >> 6, nc1 = (nr1 + 63) >> 6;
  for (int it = wave; it < nc0 + nc1; it += kVecThreads / 64) {
    const int o = it < nc0 ? 0 : 1;
    const int k = o ? k1 : k0;
    const int nr = o ? nr1 : nr0;
    const int j = (o ? it - nc0 : it) * 64 + lane;
    if (j >= nr) continue;
    const double* w = o ? w1 : w0;
    const double* Tt = fac + tk.fac[o] + j;  // T^T (nr x k, column-major): entry (j, i) at i nr + j
    double acc[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) acc[c] = 0.0;
    int i = 0;
    for (; i + kUnroll <= k; i += kUnroll) {
      double t[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) t[u] = Tt[static_cast<long long>(i + u) * nr];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const double* wr = w + (i + u) * RT;
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[c] = fma(t[u], wr[c], acc[c]);
      }
    }
    for (; i < k; ++i) {
      const double t = Tt[static_cast<long long>(i) * nr];
      const double* wr = w + i * RT;
#pragma unroll
      for (int c = 0; c < RT; ++c) acc[c] = fma(t, wr[c], acc[c]);
    }
    double* d = acc_l + ix[o * K + k + j] * RT;
#pragma unroll
    for (int c = 0; c < RT; ++c) atomicAdd(d + c, acc[c]);
  }
  __syncthreads();
  double* dst = tk.mp >= 0 ? xin : xout;
  for (int e = threadIdx.x; e < K * RT; e += kVecThreads)
    dst[(static_cast<long long>(tk.in_row) + e / RT) * R + r0 + e % RT] = acc_l[e];
}

// ------------------------------------------------------------------------------- final
// Synthesis: E = S_0 v_0, O = S_1 v_1 on rows [row0, row0+h); g(+x_i) = (E + O)/D_i at
// ring l + i and g(-x_i) = (E - O)/D_i at ring l - 1 - i (parity, Section 3.3).  One thread
// per row with both parities and all RT columns in registers; when the task has fewer row
// chunks of 64 than the work-group has waves, each chunk's contraction is split over
// several waves, whose partial sums are added in a fixed order (results do not depend on
// the schedule).
constexpr int kFinThreads = 256;
constexpr int kFinWaves = kFinThreads / 64;

template <int RT>
__global__ void __launch_bounds__(kFinThreads)
k_final_synth(const FinalTask* __restrict__ tasks, const double* __restrict__ fac,
              const double* __restrict__ v0buf, const double* __restrict__ v1buf,
              const double* __restrict__ invD, double* __restrict__ Y, int l, int R) {
  extern __shared__ double lds[];
  const FinalTask& ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1], h = ft.h;
  const int nch = (h + 63) >> 6;
  const int nparts = nch >= kFinWaves ? 1 : kFinWaves / nch;
  double* w0 = lds;
  double* w1 = lds + k0 * RT;
  double* part = w1 + k1 * RT;  // [part][row][E | O][RT] when nparts > 1
  for (int e = threadIdx.x; e < k0 * RT; e += kFinThreads)
    w0[e] = V[(static_cast<long long>(ft.in_row[0]) + e / RT) * R + r0 + e % RT];
  for (int e = threadIdx.x; e < k1 * RT; e += kFinThreads)
    w1[e] = V[(static_cast<long long>(ft.in_row[1]) + e / RT) * R + r0 + e % RT];
  __syncthreads();
  // A += S w over columns [a0, a1) of one parity (S: h x k, column-major; this thread's row)
  auto accum = [&](const double* S, const double* w, int a0, int a1, double (&A)[RT]) {
    int a = a0;
    for (; a + kUnroll <= a1; a += kUnroll) {
      double t[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) t[u] = S[static_cast<long long>(a + u) * h];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int c = 0; c < RT; ++c) A[c] = fma(t[u], w[(a + u) * RT + c], A[c]);
    }
    for (; a < a1; ++a) {
      const double t = S[static_cast<long long>(a) * h];
#pragma unroll
      for (int c = 0; c < RT; ++c) A[c] = fma(t, w[a * RT + c], A[c]);
    }
  };
  auto store = [&](int i, const double* E, const double* O) {
    const int row = ft.row0 + i;
    const double s = invD[row];
    double* yp = Y + y_row(l, ft.m, l + row) * R + r0;
    double* ym = Y + y_row(l, ft.m, l - 1 - row) * R + r0;
#pragma unroll
    for (int c = 0; c < RT; ++c) {
      yp[c] = (E[c] + O[c]) * s;
      ym[c] = (E[c] - O[c]) * s;
    }
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int it = wave; it < nch * nparts; it += kFinWaves) {
    const int ch = it / nparts, pt = it % nparts;
    const int i = ch * 64 + lane;
    if (i >= h) continue;
    double E[RT], O[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) E[c] = O[c] = 0.0;
    accum(fac + ft.fac[0] + i, w0, k0 * pt / nparts, k0 * (pt + 1) / nparts, E);
    accum(fac + ft.fac[1] + i, w1, k1 * pt / nparts, k1 * (pt + 1) / nparts, O);
    if (nparts == 1) {
      store(i, E, O);
    } else {
      double* d = part + (static_cast<long long>(pt) * h + i) * 2 * RT;
#pragma unroll
      for (int c = 0; c < RT; ++c) {
        d[c] = E[c];
        d[RT + c] = O[c];
      }
    }
  }
  if (nparts == 1) return;
  __syncthreads();
  for (int i = threadIdx.x; i < h; i += kFinThreads) {
    double E[RT], O[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) E[c] = O[c] = 0.0;
    for (int pt = 0; pt < nparts; ++pt) {
      const double* d = part + (static_cast<long long>(pt) * h + i) * 2 * RT;
#pragma unroll
      for (int c = 0; c < RT; ++c) {
        E[c] += d[c];
        O[c] += d[RT + c];
      }
    }
    store(i, E, O);
  }
}

// Transposed: v_p = S_p^T (scale * half * (G(+x) +- G(-x))): the folded rows of the task in
// LDS, one thread per output row a of either parity, summing over the task's rows.
template <int RT>
__global__ void __launch_bounds__(kFinThreads)
k_final_trans(const FinalTask* __restrict__ tasks, const double* __restrict__ fac,
              const double* __restrict__ Yin, const double* __restrict__ scale, double half,
              double* __restrict__ v0buf, double* __restrict__ v1buf, int l, int R) {
  extern __shared__ double lds[];
  const FinalTask& ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1], h = ft.h;
  double* eo0 = lds;           // h x RT, even part
  double* eo1 = lds + h * RT;  // h x RT, odd part
  for (int e = threadIdx.x; e < h * RT; e += kFinThreads) {
    const int i = e / RT, c = e % RT;
    const int row = ft.row0 + i;
    const double gp = Yin[y_row(l, ft.m, l + row) * R + r0 + c];
    const double gm = Yin[y_row(l, ft.m, l - 1 - row) * R + r0 + c];
    const double sc = scale[row] * half;
    eo0[e] = (gp + gm) * sc;
    eo1[e] = (gp - gm) * sc;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < k0 + k1; q += kFinThreads) {
    const int p = q < k0 ? 0 : 1;
    const int a = p ? q - k0 : q;
    const int k = p ? k1 : k0;
    const double* St = fac + ft.fac[p] + a;  // S^T (k x h, column-major): entry (a, i) at i k + a
    const double* src = p ? eo1 : eo0;
    double acc[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) acc[c] = 0.0;
    int i = 0;
    for (; i + kUnroll <= h; i += kUnroll) {
      double t[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) t[u] = St[static_cast<long long>(i + u) * k];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[c] = fma(t[u], src[(i + u) * RT + c], acc[c]);
    }
    for (; i < h; ++i) {
      const double t = St[static_cast<long long>(i) * k];
#pragma unroll
      for (int c = 0; c < RT; ++c) acc[c] = fma(t, src[i * RT + c], acc[c]);
    }
    double* dst = V + (static_cast<long long>(ft.in_row[p]) + a) * R + r0;
#pragma unroll
    for (int c = 0; c < RT; ++c) dst[c] = acc[c];
  }
}

// ------------------------------------------------------------------------- order maps
// Final of a per-order map A^{(m,p)} (Section 5): y = S w on the task's own output rows, with
// neither the parity unfold nor a row scaling (A carries the square roots of its weights).
// Laid out like the spherical finals above: one thread per output row (synthesis) or per
// output column of S^T (transposed), RT columns in registers, short contractions split over
// waves with fixed-order partial sums.
template <int RT>
__global__ void __launch_bounds__(kFinThreads)
k_order_final_synth(const OrderFinal* __restrict__ tasks, const double* __restrict__ fac,
                    const double* __restrict__ v0buf, const double* __restrict__ v1buf,
                    double* __restrict__ y, int R) {
  extern __shared__ double lds[];
  const OrderFinal& ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const double* V = ft.vbuf ? v1buf : v0buf;
  const int k = ft.k, h = ft.h;
  const int nch = (h + 63) >> 6;
  const int nparts = nch >= kFinWaves ? 1 : kFinWaves / nch;
  double* w = lds;           // k x RT
  double* part = w + k * RT;  // [part][row][RT] when nparts > 1
  for (int e = threadIdx.x; e < k * RT; e += kFinThreads)
    w[e] = V[(static_cast<long long>(ft.in_row) + e / RT) * R + r0 + e % RT];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int it = wave; it < nch * nparts; it += kFinWaves) {
    const int ch = it / nparts, pt = it % nparts;
    const int i = ch * 64 + lane;
    if (i >= h) continue;
    const double* S = fac + ft.fac + i;  // h x k, column-major
    double acc[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) acc[c] = 0.0;
    const int a1 = k * (pt + 1) / nparts;
    int a = k * pt / nparts;
    for (; a + kUnroll <= a1; a += kUnroll) {
      double t[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) t[u] = S[static_cast<long long>(a + u) * h];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[c] = fma(t[u], w[(a + u) * RT + c], acc[c]);
    }
    for (; a < a1; ++a) {
      const double t = S[static_cast<long long>(a) * h];
#pragma unroll
      for (int c = 0; c < RT; ++c) acc[c] = fma(t, w[a * RT + c], acc[c]);
    }
    double* d = nparts == 1 ? y + (static_cast<long long>(ft.out_row) + i) * R + r0
                            : part + (static_cast<long long>(pt) * h + i) * RT;
#pragma unroll
    for (int c = 0; c < RT; ++c) d[c] = acc[c];
  }
  if (nparts == 1) return;
  __syncthreads();
  for (int e = threadIdx.x; e < h * RT; e += kFinThreads) {
    const int i = e / RT, c = e % RT;
    double v = 0.0;
    for (int pt = 0; pt < nparts; ++pt) v += part[(static_cast<long long>(pt) * h + i) * RT + c];
    y[(static_cast<long long>(ft.out_row) + i) * R + r0 + c] = v;
  }
}

// Transposed: w = S^T y, from the transposed pool (S^T is k x h column-major there).
template <int RT>
__global__ void __launch_bounds__(kFinThreads)
k_order_final_trans(const OrderFinal* __restrict__ tasks, const double* __restrict__ fac_t,
                    const double* __restrict__ yin, double* __restrict__ v0buf,
                    double* __restrict__ v1buf, int R) {
  extern __shared__ double lds[];
  const OrderFinal& ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  double* V = ft.vbuf ? v1buf : v0buf;
  const int k = ft.k, h = ft.h;
  for (int e = threadIdx.x; e < h * RT; e += kFinThreads)
    lds[e] = yin[(static_cast<long long>(ft.out_row) + e / RT) * R + r0 + e % RT];
  __syncthreads();
  for (int a = threadIdx.x; a < k; a += kFinThreads) {
    const double* St = fac_t + ft.fac + a;  // entry (a, i) at i k + a
    double acc[RT];
#pragma unroll
    for (int c = 0; c < RT; ++c) acc[c] = 0.0;
    int i = 0;
    for (; i + kUnroll <= h; i += kUnroll) {
      double t[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) t[u] = St[static_cast<long long>(i + u) * k];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int c = 0; c < RT; ++c) acc[c] = fma(t[u], lds[(i + u) * RT + c], acc[c]);
    }
    for (; i < h; ++i) {
      const double t = St[static_cast<long long>(i) * k];
#pragma unroll
      for (int c = 0; c < RT; ++c) acc[c] = fma(t, lds[i * RT + c], acc[c]);
    }
    double* dst = V + (static_cast<long long>(ft.in_row) + a) * R + r0;
#pragma unroll
    for (int c = 0; c < RT; ++c) dst[c] = acc[c];
  }
}

// Largest column tile (<= 8) that divides R and keeps the LDS footprint of
// `per_col` doubles per column within 64 KiB.
int pick_rt(int R, long long per_col) {
  int rt = 8;
  while (rt > 1 && (R % rt != 0 || per_col * rt * 8 > 65536)) rt >>= 1;
  return rt;
}

}  // namespace

hipError_t launch_coeff_to_xin(const sht_plan_s* P, const double* coeff, double* xin, int F, int R,
                               hipStream_t s) {
  const long long ncoef = P->kind == SHT_COMPLEX ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l;
  dim3 grid(static_cast<unsigned>(P->n_pairs), 4);
  hipLaunchKernelGGL(k_coeff_to_xin, grid, dim3(kThreads), 0, s, P->d.pairs, coeff, xin, P->l, F,
                     R, P->kind, ncoef);
  return hipGetLastError();
}

hipError_t launch_xin_to_coeff(const sht_plan_s* P, const double* xin, double* coeff, int F, int R,
                               hipStream_t s) {
  const long long ncoef = P->kind == SHT_COMPLEX ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l;
  dim3 grid(static_cast<unsigned>(P->n_pairs), 4);
  hipLaunchKernelGGL(k_xin_to_coeff, grid, dim3(kThreads), 0, s, P->d.pairs, xin, coeff, P->l, F,
                     R, P->kind, ncoef);
  return hipGetLastError();
}

hipError_t launch_level(const sht_plan_s* P, int step, bool transpose, const double* in, double* out,
                        int R, int precision, hipStream_t s, double* coeff, int cls, double* xin) {
  if (mfma_ok(R)) return launch_level_mfma(P, step, transpose, in, out, R, precision, s, coeff, cls);
  if (precision != SHT_FP64) return hipErrorNotSupported;
  const long long cnt = P->step_cnt[step];
  if (cnt == 0) return hipSuccess;
  const LevelTask* tasks = P->d.tasks + P->step_off[step];
  const int K = P->step_maxK[step], k = P->step_maxk[step];
  const int RT = pick_rt(R, transpose ? K + 2 * k : K);
  if (R / RT > 65535) return hipErrorInvalidConfiguration;
  dim3 grid(static_cast<unsigned>(cnt), R / RT);
  // vectors (and, transposed, the accumulated input block) plus the two index lists
  const size_t lds = sizeof(double) * RT * (transpose ? K + 2 * k : K) + 4 * static_cast<size_t>(K) + 16;
#define LAUNCH_LEVEL(RTV)                                                                       \
  do {                                                                                           \
    if (transpose)                                                                               \
      hipLaunchKernelGGL(k_level_trans<RTV>, grid, dim3(kVecThreads), lds, s, tasks, P->d.fac_t, \
                         P->d.idx, in, out, xin, R);                                             \
    else                                                                                         \
      hipLaunchKernelGGL(k_level_synth<RTV>, grid, dim3(kVecThreads), lds, s, tasks, P->d.fac,   \
                         P->d.idx, in, xin, out, R);                                             \
  } while (0)
  switch (RT) {
    case 8: LAUNCH_LEVEL(8); break;
    case 4: LAUNCH_LEVEL(4); break;
    case 2: LAUNCH_LEVEL(2); break;
    default: LAUNCH_LEVEL(1); break;
  }
#undef LAUNCH_LEVEL
  return hipGetLastError();
}

hipError_t launch_final(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                        double* v0w, double* v1w, double* y, const double* yin, int R,
                        int precision, bool adjoint, hipStream_t s, int cls) {
  if (P->n_final == 0) return hipSuccess;
  if (mfma_ok(R))
    return launch_final_mfma(P, transpose, v0, v1, v0w, v1w, y, yin, R, precision, adjoint, s, cls);
  if (precision != SHT_FP64) return hipErrorNotSupported;
  // per column: the folded rows (transposed) or the two input blocks plus the partial sums of a
  // split contraction (at most kFinWaves parts of 64 rows, E and O)
  const long long rows = transpose ? 2LL * P->final_maxh : 2LL * P->final_maxk + 2LL * kFinThreads;
  const int RT = pick_rt(R, std::max(rows, 1LL));
  if (rows * RT * 8 > 65536 || R / RT > 65535) return hipErrorInvalidConfiguration;
  dim3 grid(static_cast<unsigned>(P->n_final), R / RT);
  const size_t lds = sizeof(double) * RT * std::max(rows, 1LL);
  const double* scale = adjoint ? P->d.invD : P->d.D;
  const double half = adjoint ? 1.0 : 0.5;
#define LAUNCH_FINAL(RTV)                                                                       \
  do {                                                                                           \
    if (transpose)                                                                               \
      hipLaunchKernelGGL(k_final_trans<RTV>, grid, dim3(kFinThreads), lds, s, P->d.finals,        \
                         P->d.fac_t, yin, scale, half, v0w, v1w, P->l, R);                       \
    else                                                                                         \
      hipLaunchKernelGGL(k_final_synth<RTV>, grid, dim3(kFinThreads), lds, s, P->d.finals,        \
                         P->d.fac, v0, v1, P->d.invD, y, P->l, R);                               \
  } while (0)
  switch (RT) {
    case 8: LAUNCH_FINAL(8); break;
    case 4: LAUNCH_FINAL(4); break;
    case 2: LAUNCH_FINAL(2); break;
    default: LAUNCH_FINAL(1); break;
  }
#undef LAUNCH_FINAL
  return hipGetLastError();
}

hipError_t launch_order_final(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                              double* v0w, double* v1w, double* y, const double* yin, int R, hipStream_t s) {
  if (P->n_ofinal == 0) return hipSuccess;
  // per column: the staged rows (transposed) or the input block plus split partial sums
  const long long rows = transpose ? std::max(1, P->ofinal_maxh) : P->ofinal_maxk + kFinThreads;
  const int RT = pick_rt(R, rows);
  if (rows * RT * 8 > 65536 || R / RT > 65535) return hipErrorInvalidConfiguration;
  dim3 grid(static_cast<unsigned>(P->n_ofinal), R / RT);
  const size_t lds = sizeof(double) * RT * rows;
#define LAUNCH_OFINAL(RTV)                                                                           \
  do {                                                                                                \
    if (transpose)                                                                                    \
      hipLaunchKernelGGL(k_order_final_trans<RTV>, grid, dim3(kFinThreads), lds, s, P->d.ofinals,     \
                         P->d.fac_t, yin, v0w, v1w, R);                                               \
    else                                                                                              \
      hipLaunchKernelGGL(k_order_final_synth<RTV>, grid, dim3(kFinThreads), lds, s, P->d.ofinals,     \
                         P->d.fac, v0, v1, y, R);                                                     \
  } while (0)
  switch (RT) {
    case 8: LAUNCH_OFINAL(8); break;
    case 4: LAUNCH_OFINAL(4); break;
    case 2: LAUNCH_OFINAL(2); break;
    default: LAUNCH_OFINAL(1); break;
  }
#undef LAUNCH_OFINAL
  return hipGetLastError();
}

}  // namespace sht
