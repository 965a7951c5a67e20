// Longitude sums by FFT (Section 2: the sums over m of equation
// (alternate_expansion) are discrete Fourier transforms).  One work-group owns one
// (field, ring) row of N = 4l points, held in LDS; radix-2 decimation in time after a
// bit-reversed load.  FP64 throughout.
//
// Synthesis reads the Legendre output Y[m][ring][R] (bins +m and -m = N - m) and writes
// the grid row; analysis reads a grid row and writes the bins back in the same layout,
// scaled by 1/N (analysis) or 1 (adjoint).
#include "sht_internal.h"

namespace sht {

namespace {

constexpr int kFftThreads = 256;

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) {
  return __brev(v) >> (32 - bits);
}

// In-place radix-2 DIT on bit-reversed input; sign +1 uses e^{+i}, -1 uses e^{-i}.
__device__ void fft_lds(double2* X, int N, int logN, const double* __restrict__ tw, double sign) {
  for (int s = 0; s < logN; ++s) {
    const int half = 1 << s;
    const int stride = N >> (s + 1);  // twiddle index step
    __syncthreads();
    for (int b = threadIdx.x; b < N / 2; b += kFftThreads) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> s) << (s + 1)) + pos;
      const int i1 = i0 + half;
      const int q = pos * stride;
      const double wr = tw[2 * q], wi = sign * tw[2 * q + 1];
      const double2 a = X[i0], c = X[i1];
      const double br = c.x * wr - c.y * wi;
      const double bi = c.x * wi + c.y * wr;
      X[i0] = make_double2(a.x + br, a.y + bi);
      X[i1] = make_double2(a.x - br, a.y - bi);
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kFftThreads)
k_fft_synth(const double* __restrict__ Y, double* __restrict__ grid, const double* __restrict__ tw,
            int l, int R, int kind) {
  extern __shared__ double2 X[];
  const int ring = blockIdx.x;
  const int f = blockIdx.y;
  const int L2 = 2 * l;
  const int N = 4 * l;
  int logN = 0;
  while ((1 << logN) < N) ++logN;
  for (int b = threadIdx.x; b < N; b += kFftThreads) {
    double2 v = make_double2(0.0, 0.0);
    if (b < L2) {
      const long long row = static_cast<long long>(b) * L2 + ring;
      const double* src = Y + row * R + (kind == SHT_COMPLEX ? 4 * f : 2 * f);
      v = make_double2(src[0], src[1]);
    } else if (b > L2) {
      const int m = N - b;
      const long long row = static_cast<long long>(m) * L2 + ring;
      if (kind == SHT_COMPLEX) {
        const double* src = Y + row * R + 4 * f + 2;
        v = make_double2(src[0], src[1]);
      } else {
        const double* src = Y + row * R + 2 * f;
        v = make_double2(src[0], -src[1]);  // g_{-m} = conj(g_m) for real fields
      }
    }
    X[bitrev(b, logN)] = v;
  }
  fft_lds(X, N, logN, tw, 1.0);
  const long long rowbase = (static_cast<long long>(f) * L2 + ring) * N;
  if (kind == SHT_COMPLEX) {
    double2* out = reinterpret_cast<double2*>(grid) + rowbase;
    for (int j = threadIdx.x; j < N; j += kFftThreads) out[j] = X[j];
  } else {
    for (int j = threadIdx.x; j < N; j += kFftThreads) grid[rowbase + j] = X[j].x;
  }
}

__global__ void __launch_bounds__(kFftThreads)
k_fft_analyze(const double* __restrict__ grid, double* __restrict__ Y, const double* __restrict__ tw,
              int l, int R, int kind, double scale, double real_pos) {
  extern __shared__ double2 X[];
  const int ring = blockIdx.x;
  const int f = blockIdx.y;
  const int L2 = 2 * l;
  const int N = 4 * l;
  int logN = 0;
  while ((1 << logN) < N) ++logN;
  const long long rowbase = (static_cast<long long>(f) * L2 + ring) * N;
  for (int j = threadIdx.x; j < N; j += kFftThreads) {
    double2 v;
    if (kind == SHT_COMPLEX)
      v = reinterpret_cast<const double2*>(grid)[rowbase + j];
    else
      v = make_double2(grid[rowbase + j], 0.0);
    X[bitrev(j, logN)] = v;
  }
  fft_lds(X, N, logN, tw, -1.0);
  for (int m = threadIdx.x; m < L2; m += kFftThreads) {
    const long long row = static_cast<long long>(m) * L2 + ring;
    if (kind == SHT_COMPLEX) {
      double* dst = Y + row * R + 4 * f;
      const double2 p = X[m];
      dst[0] = p.x * scale;
      dst[1] = p.y * scale;
      if (m > 0) {
        const double2 q = X[N - m];
        dst[2] = q.x * scale;
        dst[3] = q.y * scale;
      } else {
        dst[2] = 0.0;
        dst[3] = 0.0;
      }
    } else {
      // real fields store m >= 0 only; m > 0 stands for the pair +-m (factor real_pos)
      double* dst = Y + row * R + 2 * f;
      const double2 p = X[m];
      const double sc = m > 0 ? scale * real_pos : scale;
      dst[0] = p.x * sc;
      dst[1] = p.y * sc;
    }
  }
}

}  // namespace

static hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

hipError_t launch_fft_synth(const sht_plan_s* P, const double* y, double* grid, int F, int R,
                            hipStream_t s) {
  const int N = 4 * P->l;
  dim3 gridd(2 * P->l, F);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_synth), sizeof(double2) * N);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fft_synth, gridd, dim3(kFftThreads), sizeof(double2) * N, s, y, grid,
                     P->d.twiddle, P->l, R, P->kind);
  return hipGetLastError();
}

hipError_t launch_fft_analyze(const sht_plan_s* P, const double* grid, double* y, int F, int R,
                              double scale, double real_pos, hipStream_t s) {
  const int N = 4 * P->l;
  dim3 gridd(2 * P->l, F);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_analyze), sizeof(double2) * N);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fft_analyze, gridd, dim3(kFftThreads), sizeof(double2) * N, s, grid, y,
                     P->d.twiddle, P->l, R, P->kind, scale, real_pos);
  return hipGetLastError();
}

}  // namespace sht
