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
// Synthesis: out_o = in[skel_o] + T_o in[red_o] for the task's one or two outputs.
// Tasks whose input rows are coefficients (mp >= 0: leaves, level-1 tasks over folded
// leaves) read them from the internal coefficient rows `xin` instead of `in`.
template <int RT>
__global__ void __launch_bounds__(kThreads)
k_level_synth(const LevelTask* __restrict__ tasks, const double* __restrict__ fac,
              const uint16_t* __restrict__ idx, const double* __restrict__ in,
              const double* __restrict__ xin, double* __restrict__ out, int R) {
  extern __shared__ double lds[];
  const LevelTask tk = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const int K = tk.K;
  const double* src = tk.mp >= 0 ? xin : in;
  for (int e = threadIdx.x; e < K * RT; e += kThreads) {
    const int row = e / RT, c = e % RT;
    lds[e] = src[(static_cast<long long>(tk.in_row) + row) * R + r0 + c];
  }
  __syncthreads();
  for (int o = 0; o < 2; ++o) {
    const int k = tk.k[o];
    if (k <= 0) continue;
    const uint16_t* skel = idx + tk.idx[o];
    const uint16_t* red = skel + k;
    const int nr = K - k;
    const double* T = fac + tk.fac[o];
    for (int e = threadIdx.x; e < k * RT; e += kThreads) {
      const int i = e / RT, c = e % RT;
      double acc = lds[skel[i] * RT + c];
      for (int j = 0; j < nr; ++j) acc = fma(T[static_cast<long long>(j) * k + i], lds[red[j] * RT + c], acc);
      out[(static_cast<long long>(tk.out_row[o]) + i) * R + r0 + c] = acc;
    }
  }
}

// Transposed: in = sum_o (Ã_o)^T out_o, where Ã_o has the identity at skel_o and T_o at
// red_o.  Each input row receives exactly one term from each output block.
template <int RT>
__global__ void __launch_bounds__(kThreads)
k_level_trans(const LevelTask* __restrict__ tasks, const double* __restrict__ fac,
              const uint16_t* __restrict__ idx, const double* __restrict__ win,
              double* __restrict__ xout, double* __restrict__ xin, int R) {
  extern __shared__ double lds[];
  const LevelTask tk = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const int K = tk.K;
  const int k0 = tk.k[0];
  const int k1 = tk.k[1] < 0 ? 0 : tk.k[1];
  double* w0 = lds;
  double* w1 = w0 + k0 * RT;
  double* acc = w1 + k1 * RT;
  for (int e = threadIdx.x; e < k0 * RT; e += kThreads) {
    const int row = e / RT, c = e % RT;
    w0[e] = win[(static_cast<long long>(tk.out_row[0]) + row) * R + r0 + c];
  }
  for (int e = threadIdx.x; e < k1 * RT; e += kThreads) {
    const int row = e / RT, c = e % RT;
    w1[e] = win[(static_cast<long long>(tk.out_row[1]) + row) * R + r0 + c];
  }
  __syncthreads();
  const int nouts = tk.k[1] < 0 ? 1 : 2;
  for (int o = 0; o < nouts; ++o) {
    const int k = o ? k1 : k0;
    const double* w = o ? w1 : w0;
    const uint16_t* skel = idx + tk.idx[o];
    const uint16_t* red = skel + k;
    const double* T = fac + tk.fac[o];
    for (int e = threadIdx.x; e < K * RT; e += kThreads) {
      const int q = e / RT, c = e % RT;
      int dst;
      double v;
      if (q < k) {
        dst = skel[q];
        v = w[q * RT + c];
      } else {
        // T^T stored column-major (nr x k): entry (j, i) at i * nr + j
        const int j = q - k;
        const int nr = K - k;
        dst = red[j];
        v = 0.0;
        for (int i = 0; i < k; ++i) v = fma(T[static_cast<long long>(i) * nr + j], w[i * RT + c], v);
      }
      if (o == 0)
        acc[dst * RT + c] = v;
      else
        acc[dst * RT + c] += v;
    }
    __syncthreads();
  }
  double* dst = tk.mp >= 0 ? xin : xout;
  for (int e = threadIdx.x; e < K * RT; e += kThreads) {
    const int row = e / RT, c = e % RT;
    dst[(static_cast<long long>(tk.in_row) + row) * R + r0 + c] = acc[e];
  }
}

// ------------------------------------------------------------------------------- final
// Synthesis: E = S_0 v_0, O = S_1 v_1 on rows [row0, row0+h); g(+x_i) = (E + O)/D_i at
// ring l + i and g(-x_i) = (E - O)/D_i at ring l - 1 - i (parity, Section 3.3).
template <int RT>
__global__ void __launch_bounds__(kThreads)
k_final_synth(const FinalTask* __restrict__ tasks, const double* __restrict__ fac,
              const double* __restrict__ v0buf, const double* __restrict__ v1buf,
              const double* __restrict__ invD, double* __restrict__ Y, int l, int R) {
  extern __shared__ double lds[];
  const FinalTask ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1];
  double* w0 = lds;
  double* w1 = lds + k0 * RT;
  for (int e = threadIdx.x; e < k0 * RT; e += kThreads)
    w0[e] = V[(static_cast<long long>(ft.in_row[0]) + e / RT) * R + r0 + e % RT];
  for (int e = threadIdx.x; e < k1 * RT; e += kThreads)
    w1[e] = V[(static_cast<long long>(ft.in_row[1]) + e / RT) * R + r0 + e % RT];
  __syncthreads();
  const int h = ft.h;
  const double* S0 = fac + ft.fac[0];
  const double* S1 = fac + ft.fac[1];
  for (int e = threadIdx.x; e < h * RT; e += kThreads) {
    const int i = e / RT, c = e % RT;
    double E = 0.0, O = 0.0;
    for (int a = 0; a < k0; ++a) E = fma(S0[static_cast<long long>(a) * h + i], w0[a * RT + c], E);
    for (int a = 0; a < k1; ++a) O = fma(S1[static_cast<long long>(a) * h + i], w1[a * RT + c], O);
    const int row = ft.row0 + i;
    const double s = invD[row];
    Y[y_row(l, ft.m, l + row) * R + r0 + c] = (E + O) * s;
    Y[y_row(l, ft.m, l - 1 - row) * R + r0 + c] = (E - O) * s;
  }
}

// Transposed: v_p = S_p^T (scale * half * (G(+x) +- G(-x))).
template <int RT>
__global__ void __launch_bounds__(kThreads)
k_final_trans(const FinalTask* __restrict__ tasks, const double* __restrict__ fac,
              const double* __restrict__ Yin, const double* __restrict__ scale, double half,
              double* __restrict__ v0buf, double* __restrict__ v1buf, int l, int R) {
  constexpr int ICH = 64;
  constexpr int NACC = 8;
  __shared__ double eo[2][ICH * RT];
  const FinalTask ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1];
  const int nout = (k0 + k1) * RT;
  const int h = ft.h;
  const double* S0 = fac + ft.fac[0];
  const double* S1 = fac + ft.fac[1];
  for (int g0 = 0; g0 < nout; g0 += kThreads * NACC) {
    double accv[NACC];
#pragma unroll
    for (int u = 0; u < NACC; ++u) accv[u] = 0.0;
    for (int i0 = 0; i0 < h; i0 += ICH) {
      const int ih = min(ICH, h - i0);
      __syncthreads();
      for (int e = threadIdx.x; e < ih * RT; e += kThreads) {
        const int i = e / RT, c = e % RT;
        const int row = ft.row0 + i0 + i;
        const double gp = Yin[y_row(l, ft.m, l + row) * R + r0 + c];
        const double gm = Yin[y_row(l, ft.m, l - 1 - row) * R + r0 + c];
        const double sc = scale[row] * half;
        eo[0][e] = (gp + gm) * sc;
        eo[1][e] = (gp - gm) * sc;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NACC; ++u) {
        const int e = g0 + u * kThreads + threadIdx.x;
        if (e >= nout) continue;
        const int q = e / RT, c = e % RT;
        const int p = q < k0 ? 0 : 1;
        const int a = p ? q - k0 : q;
        // S^T stored column-major (k x h): entry (a, i) at i * k + a
        const int kp = p ? k1 : k0;
        const double* Sa = (p ? S1 : S0) + static_cast<long long>(i0) * kp + a;
        const double* src = eo[p];
        double v = accv[u];
        for (int i = 0; i < ih; ++i) v = fma(Sa[static_cast<long long>(i) * kp], src[i * RT + c], v);
        accv[u] = v;
      }
    }
#pragma unroll
    for (int u = 0; u < NACC; ++u) {
      const int e = g0 + u * kThreads + threadIdx.x;
      if (e >= nout) continue;
      const int q = e / RT, c = e % RT;
      const int p = q < k0 ? 0 : 1;
      const int a = p ? q - k0 : q;
      V[(static_cast<long long>(ft.in_row[p]) + a) * R + r0 + c] = accv[u];
    }
  }
}

// ------------------------------------------------------------------------- order maps
// Final of a per-order map A^{(m,p)} (Section 5): y = S w on the task's own output rows, with
// neither the parity unfold nor a row scaling (A carries the square roots of its weights).
template <int RT>
__global__ void __launch_bounds__(kThreads)
k_order_final_synth(const OrderFinal* __restrict__ tasks, const double* __restrict__ fac,
                    const double* __restrict__ v0buf, const double* __restrict__ v1buf,
                    double* __restrict__ y, int R) {
  extern __shared__ double lds[];
  const OrderFinal ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  const double* V = ft.vbuf ? v1buf : v0buf;
  const int k = ft.k, h = ft.h;
  for (int e = threadIdx.x; e < k * RT; e += kThreads)
    lds[e] = V[(static_cast<long long>(ft.in_row) + e / RT) * R + r0 + e % RT];
  __syncthreads();
  const double* S = fac + ft.fac;  // h x k, column-major
  for (int e = threadIdx.x; e < h * RT; e += kThreads) {
    const int i = e / RT, c = e % RT;
    double acc = 0.0;
    for (int a = 0; a < k; ++a) acc = fma(S[static_cast<long long>(a) * h + i], lds[a * RT + c], acc);
    y[(static_cast<long long>(ft.out_row) + i) * R + r0 + c] = acc;
  }
}

// Transposed: w = S^T y, from the transposed pool (S^T is k x h column-major there).
template <int RT>
__global__ void __launch_bounds__(kThreads)
k_order_final_trans(const OrderFinal* __restrict__ tasks, const double* __restrict__ fac_t,
                    const double* __restrict__ yin, double* __restrict__ v0buf,
                    double* __restrict__ v1buf, int R) {
  extern __shared__ double lds[];
  const OrderFinal ft = tasks[blockIdx.x];
  const int r0 = blockIdx.y * RT;
  double* V = ft.vbuf ? v1buf : v0buf;
  const int k = ft.k, h = ft.h;
  for (int e = threadIdx.x; e < h * RT; e += kThreads)
    lds[e] = yin[(static_cast<long long>(ft.out_row) + e / RT) * R + r0 + e % RT];
  __syncthreads();
  const double* St = fac_t + ft.fac;
  for (int e = threadIdx.x; e < k * RT; e += kThreads) {
    const int a = e / RT, c = e % RT;
    double acc = 0.0;
    for (int i = 0; i < h; ++i) acc = fma(St[static_cast<long long>(i) * k + a], lds[i * RT + c], acc);
    V[(static_cast<long long>(ft.in_row) + a) * R + r0 + c] = acc;
  }
}

// Largest column tile (<= 16) that divides R and keeps the LDS footprint of
// `per_col` doubles per column within 64 KiB.
int pick_rt(int R, long long per_col) {
  int rt = 16;
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
  dim3 grid(static_cast<unsigned>(cnt), R / RT);
  const size_t lds = transpose ? sizeof(double) * RT * (K + 2 * k) : sizeof(double) * RT * K;
#define LAUNCH_LEVEL(RTV)                                                                       \
  do {                                                                                           \
    if (transpose)                                                                               \
      hipLaunchKernelGGL(k_level_trans<RTV>, grid, dim3(kThreads), lds, s, tasks, P->d.fac_t,    \
                         P->d.idx, in, out, xin, R);                                             \
    else                                                                                         \
      hipLaunchKernelGGL(k_level_synth<RTV>, grid, dim3(kThreads), lds, s, tasks, P->d.fac,      \
                         P->d.idx, in, xin, out, R);                                             \
  } while (0)
  switch (RT) {
    case 16: LAUNCH_LEVEL(16); break;
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
  const int RT = pick_rt(R, std::max(2LL * P->final_maxk, 64LL * 2));
  dim3 grid(static_cast<unsigned>(P->n_final), R / RT);
  const size_t lds = sizeof(double) * RT * 2 * P->final_maxk;
  const double* scale = adjoint ? P->d.invD : P->d.D;
  const double half = adjoint ? 1.0 : 0.5;
#define LAUNCH_FINAL(RTV)                                                                       \
  do {                                                                                           \
    if (transpose)                                                                               \
      hipLaunchKernelGGL(k_final_trans<RTV>, grid, dim3(kThreads), 0, s, P->d.finals, P->d.fac_t,\
                         yin, scale, half, v0w, v1w, P->l, R);                                   \
    else                                                                                         \
      hipLaunchKernelGGL(k_final_synth<RTV>, grid, dim3(kThreads), lds, s, P->d.finals,          \
                         P->d.fac, v0, v1, P->d.invD, y, P->l, R);                               \
  } while (0)
  switch (RT) {
    case 16: LAUNCH_FINAL(16); break;
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
  const long long rows = std::max(1, transpose ? P->ofinal_maxh : P->ofinal_maxk);
  const int RT = pick_rt(R, rows);
  if (rows * RT * 8 > 65536 || R / RT > 65535) return hipErrorInvalidConfiguration;
  dim3 grid(static_cast<unsigned>(P->n_ofinal), R / RT);
  const size_t lds = sizeof(double) * RT * rows;
#define LAUNCH_OFINAL(RTV)                                                                           \
  do {                                                                                                \
    if (transpose)                                                                                    \
      hipLaunchKernelGGL(k_order_final_trans<RTV>, grid, dim3(kThreads), lds, s, P->d.ofinals,        \
                         P->d.fac_t, yin, v0w, v1w, R);                                               \
    else                                                                                              \
      hipLaunchKernelGGL(k_order_final_synth<RTV>, grid, dim3(kThreads), lds, s, P->d.ofinals,        \
                         P->d.fac, v0, v1, y, R);                                                     \
  } while (0)
  switch (RT) {
    case 16: LAUNCH_OFINAL(16); break;
    case 8: LAUNCH_OFINAL(8); break;
    case 4: LAUNCH_OFINAL(4); break;
    case 2: LAUNCH_OFINAL(2); break;
    default: LAUNCH_OFINAL(1); break;
  }
#undef LAUNCH_OFINAL
  return hipGetLastError();
}

}  // namespace sht
