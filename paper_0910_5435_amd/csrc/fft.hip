// Longitude sums by FFT (Section 2: the sums over m of equation
// (alternate_expansion) are discrete Fourier transforms).  One work-group owns one
// (field, ring) row of N = 4l points, held in LDS; decimation in time after a
// bit-reversed load, two radix-2 stages per LDS pass (each thread owns a closed set of
// four points), FP64 throughout.
//
// Synthesis reads the Legendre output Y[ring][m][R] (bins +m and -m = N - m) and writes
// the grid row; analysis reads a grid row and writes the bins back in the same layout,
// scaled by 1/N (analysis) or 1 (adjoint).  A Y row holds all fields of one (ring, m),
// so work-groups are numbered field-fastest within each XCD: the groups of one ring run
// together on one XCD and share the L2 lines of their Y gathers and scatters, all within
// that ring's contiguous block of Y.
#include <atomic>

#include "sht_internal.h"

namespace sht {

namespace {

constexpr int kFftThreads = 1024;
constexpr int kBatch = 2;  // global loads in flight per thread while staging a row
constexpr int kXcd = 8;

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) { return __brev(v) >> (32 - bits); }

inline size_t fft_lds_bytes(int N) { return sizeof(double2) * static_cast<size_t>(N); }

__device__ __forceinline__ double2 cmul(double2 a, double wr, double wi) {
  return make_double2(a.x * wr - a.y * wi, a.x * wi + a.y * wr);
}

// In-place DIT on a bit-reversed row; sign +1 uses e^{+i}, -1 uses e^{-i}.
__device__ void fft_lds(double2* X, int N, int logN, const double* __restrict__ tw, double sign) {
  int s = 0;
  for (; s + 1 < logN; s += 2) {
    const int h = 1 << s;
    __syncthreads();
    for (int b = threadIdx.x; b < N / 4; b += kFftThreads) {
      const int pos = b & (h - 1);
      const int i0 = ((b >> s) << (s + 2)) + pos;
      // stage s: pairs (i0, i0+h), (i0+2h, i0+3h), twiddle e^{i pi pos / h}
      const int q1 = pos * (N >> (s + 1));
      const double w1r = tw[2 * q1], w1i = sign * tw[2 * q1 + 1];
      // stage s+1: pairs (i0, i0+2h) with e^{i pi pos/(2h)}, (i0+h, i0+3h) with e^{i pi (pos+h)/(2h)}
      const int q2 = pos * (N >> (s + 2));
      const int q3 = (pos + h) * (N >> (s + 2));
      const double w2r = tw[2 * q2], w2i = sign * tw[2 * q2 + 1];
      const double w3r = tw[2 * q3], w3i = sign * tw[2 * q3 + 1];
      const double2 x0 = X[i0], x1 = cmul(X[i0 + h], w1r, w1i);
      const double2 x2 = X[i0 + 2 * h], x3 = cmul(X[i0 + 3 * h], w1r, w1i);
      const double2 a0 = make_double2(x0.x + x1.x, x0.y + x1.y);
      const double2 a1 = make_double2(x0.x - x1.x, x0.y - x1.y);
      const double2 a2 = cmul(make_double2(x2.x + x3.x, x2.y + x3.y), w2r, w2i);
      const double2 a3 = cmul(make_double2(x2.x - x3.x, x2.y - x3.y), w3r, w3i);
      X[i0] = make_double2(a0.x + a2.x, a0.y + a2.y);
      X[i0 + 2 * h] = make_double2(a0.x - a2.x, a0.y - a2.y);
      X[i0 + h] = make_double2(a1.x + a3.x, a1.y + a3.y);
      X[i0 + 3 * h] = make_double2(a1.x - a3.x, a1.y - a3.y);
    }
  }
  if (s < logN) {  // one radix-2 stage left
    const int h = 1 << s;
    __syncthreads();
    for (int b = threadIdx.x; b < N / 2; b += kFftThreads) {
      const int pos = b & (h - 1);
      const int i0 = ((b >> s) << (s + 1)) + pos;
      const int q = pos * (N >> (s + 1));
      const double wr = tw[2 * q], wi = sign * tw[2 * q + 1];
      const double2 a = X[i0], c = cmul(X[i0 + h], wr, wi);
      X[i0] = make_double2(a.x + c.x, a.y + c.y);
      X[i0 + h] = make_double2(a.x - c.x, a.y - c.y);
    }
  }
  __syncthreads();
}

// (ring, field) of this work-group: fields fastest within an XCD.
__device__ __forceinline__ bool ring_field(int rings, int F, int& ring, int& f) {
  const long long id = blockIdx.x;
  const int xcd = static_cast<int>(id % kXcd);
  const long long slot = id / kXcd;
  const long long per = (static_cast<long long>(rings) * F + kXcd - 1) / kXcd;
  const long long lin = xcd * per + slot;  // contiguous range of (ring, field) per XCD
  if (slot >= per || lin >= static_cast<long long>(rings) * F) return false;
  ring = static_cast<int>(lin / F);
  f = static_cast<int>(lin % F);
  return true;
}

// Base of field f's grid: the f-th block of a contiguous [field][ring][phi] array, or the
// f-th entry of a per-field pointer table.
__device__ __forceinline__ double* field_grid(double* grid, double* const* fptr, int f, int l, int kind) {
  if (fptr) return fptr[f];
  return grid + static_cast<long long>(f) * (2LL * l) * (4LL * l) * (kind == SHT_COMPLEX ? 2 : 1);
}

// One thread per order m: the bins +m and -m of the field sit next to each other in the Y
// row (ring, m), so they are read together.
__global__ void __launch_bounds__(kFftThreads)
k_fft_synth(const double* __restrict__ Y, double* __restrict__ grid, double* const* __restrict__ fptr,
            const double* __restrict__ tw, int l, int R, int F, int kind) {
  extern __shared__ double2 X[];
  const int L2 = 2 * l;
  int ring, f;
  if (!ring_field(L2, F, ring, f)) return;
  const int N = 4 * l;
  const int logN = 31 - __clz(N);
  const int w = kind == SHT_COMPLEX ? 4 : 2;  // Y words per field
  // m = 0 .. 2l-1; the bin 2l (order 2l is outside the band) is zero
  for (int m0 = threadIdx.x; m0 < L2; m0 += kFftThreads * kBatch) {
    double2 v[kBatch][2];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int m = m0 + u * kFftThreads;
      v[u][0] = v[u][1] = make_double2(0.0, 0.0);
      if (m < L2) {
        const double* src = Y + y_row(l, m, ring) * R + w * f;
        v[u][0] = *reinterpret_cast<const double2*>(src);
        if (kind == SHT_COMPLEX)
          v[u][1] = *reinterpret_cast<const double2*>(src + 2);
        else
          v[u][1] = make_double2(v[u][0].x, -v[u][0].y);  // g_{-m} = conj(g_m) for real fields
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int m = m0 + u * kFftThreads;
      if (m < L2) {
        X[bitrev(m, logN)] = v[u][0];
        if (m > 0) X[bitrev(N - m, logN)] = v[u][1];
      }
    }
  }
  if (threadIdx.x == 0) X[bitrev(L2, logN)] = make_double2(0.0, 0.0);
  fft_lds(X, N, logN, tw, 1.0);
  double* gb = field_grid(grid, fptr, f, l, kind);
  const long long rowbase = static_cast<long long>(ring) * N;
  if (kind == SHT_COMPLEX) {
    double2* out = reinterpret_cast<double2*>(gb) + rowbase;
    for (int j = threadIdx.x; j < N; j += kFftThreads) out[j] = X[j];
  } else {
    for (int j = threadIdx.x; j < N; j += kFftThreads) gb[rowbase + j] = X[j].x;
  }
}

__global__ void __launch_bounds__(kFftThreads)
k_fft_analyze(const double* __restrict__ grid, double* const* __restrict__ fptr, double* __restrict__ Y,
              const double* __restrict__ tw, int l, int R, int F, int kind, double scale, double real_pos) {
  extern __shared__ double2 X[];
  const int L2 = 2 * l;
  int ring, f;
  if (!ring_field(L2, F, ring, f)) return;
  const int N = 4 * l;
  const int logN = 31 - __clz(N);
  const double* gb = field_grid(const_cast<double*>(grid), fptr, f, l, kind);
  const long long rowbase = static_cast<long long>(ring) * N;
  for (int j0 = threadIdx.x; j0 < N; j0 += kFftThreads * kBatch) {
    double2 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int j = j0 + u * kFftThreads;
      if (j >= N)
        v[u] = make_double2(0.0, 0.0);
      else if (kind == SHT_COMPLEX)
        v[u] = reinterpret_cast<const double2*>(gb)[rowbase + j];
      else
        v[u] = make_double2(gb[rowbase + j], 0.0);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int j = j0 + u * kFftThreads;
      if (j < N) X[bitrev(j, logN)] = v[u];
    }
  }
  fft_lds(X, N, logN, tw, -1.0);
  for (int m = threadIdx.x; m < L2; m += kFftThreads) {
    const long long row = y_row(l, m, ring);
    if (kind == SHT_COMPLEX) {
      double* dst = Y + row * R + 4 * f;
      const double2 p = X[m];
      const double2 q = m > 0 ? X[N - m] : make_double2(0.0, 0.0);
      *reinterpret_cast<double2*>(dst) = make_double2(p.x * scale, p.y * scale);
      *reinterpret_cast<double2*>(dst + 2) = make_double2(q.x * scale, q.y * scale);
    } else {
      // real fields store m >= 0 only; m > 0 stands for the pair +-m (factor real_pos)
      const double2 p = X[m];
      const double sc = m > 0 ? scale * real_pos : scale;
      *reinterpret_cast<double2*>(Y + row * R + 2 * f) = make_double2(p.x * sc, p.y * sc);
    }
  }
}

// Raises a kernel's dynamic-LDS limit once per size (so that launches recorded into a graph
// make no attribute calls after fft_prepare).
std::atomic<size_t> g_lds_synth{65536}, g_lds_analyze{65536};

hipError_t allow_lds_fft(const void* fn, size_t bytes) {
  std::atomic<size_t>& done = fn == reinterpret_cast<const void*>(&k_fft_synth) ? g_lds_synth : g_lds_analyze;
  if (bytes <= done.load()) return hipSuccess;
  const hipError_t e =
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  if (e == hipSuccess) {
    size_t cur = done.load();
    while (cur < bytes && !done.compare_exchange_weak(cur, bytes)) {
    }
  }
  return e;
}

unsigned fft_grid(int l, int F) {
  const long long per = (2LL * l * F + kXcd - 1) / kXcd;
  return static_cast<unsigned>(per * kXcd);
}

}  // namespace

hipError_t fft_prepare(int l) {
  const size_t bytes = fft_lds_bytes(4 * l);
  hipError_t e = allow_lds_fft(reinterpret_cast<const void*>(&k_fft_synth), bytes);
  if (e == hipSuccess) e = allow_lds_fft(reinterpret_cast<const void*>(&k_fft_analyze), bytes);
  return e;
}

hipError_t launch_fft_synth(const sht_plan_s* P, const double* y, double* grid, int F, int R,
                            hipStream_t s, double* const* fptr) {
  const int N = 4 * P->l;
  hipError_t e = allow_lds_fft(reinterpret_cast<const void*>(&k_fft_synth), fft_lds_bytes(N));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fft_synth, dim3(fft_grid(P->l, F)), dim3(kFftThreads), fft_lds_bytes(N), s,
                     y, grid, fptr, P->d.twiddle, P->l, R, F, P->kind);
  return hipGetLastError();
}

hipError_t launch_fft_analyze(const sht_plan_s* P, const double* grid, double* y, int F, int R,
                              double scale, double real_pos, hipStream_t s, double* const* fptr) {
  const int N = 4 * P->l;
  hipError_t e = allow_lds_fft(reinterpret_cast<const void*>(&k_fft_analyze), fft_lds_bytes(N));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fft_analyze, dim3(fft_grid(P->l, F)), dim3(kFftThreads), fft_lds_bytes(N), s,
                     grid, fptr, y, P->d.twiddle, P->l, R, F, P->kind, scale, real_pos);
  return hipGetLastError();
}

}  // namespace sht
