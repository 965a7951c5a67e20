// Helpers shared by the matrix-core apply kernels (the FP64 / split-FP32 / FP32 forms and
// the int8-slice form): XCD-aware work-group numbering, staged LDS loads of vector blocks,
// and the leaf gather from the caller's coefficient layout.
#pragma once

#include <hip/hip_runtime.h>

#include "sht_internal.h"

namespace sht {
namespace {

constexpr int kXcd = 8;

// (task, column block) of this work-group under the XCD-aware numbering; false if padding.
__device__ __forceinline__ bool xcd_map(long long ntasks, int nblk, long long& task, int& blk) {
  const long long id = blockIdx.x;
  const int xcd = static_cast<int>(id % kXcd);
  const long long slot = id / kXcd;
  task = (slot / nblk) * kXcd + xcd;
  blk = static_cast<int>(slot % nblk);
  return task < ntasks;
}

inline unsigned xcd_grid(long long ntasks, int nblk) {
  return static_cast<unsigned>(((ntasks + kXcd - 1) / kXcd) * kXcd * nblk);
}

// LDS row stride (doubles) for NT columns: a 16-byte skew spreads the four rows a B
// fragment touches over different banks.
template <int NT>
constexpr int ldp() { return NT + 2; }

// Address of row j, local column col of a leaf block in the caller's coefficients; null if
// there is no such entry (the -m half at m = 0, padding).  imag0: the imaginary part at
// m = 0 of a real field, which reads as 0 and is written as 0.
__device__ __forceinline__ double* leaf_ptr(const CoefIO& io, int m, int p, int j0, int j, long long col,
                                            bool& imag0) {
  const int k = m + p + 2 * (j0 + j);
  const int cc = static_cast<int>(col & 1);
  imag0 = false;
  if (io.kind == SHT_COMPLEX) {
    const int f = static_cast<int>(col >> 2), s = static_cast<int>((col >> 1) & 1);
    return (m == 0 && s == 1) ? nullptr : io.at(f, m, s, k, cc);
  }
  const int f = static_cast<int>(col >> 1);
  imag0 = m == 0 && cc == 1;
  return io.at(f, m, 0, k, cc);
}

// Visits the K x NT block of a leaf task in an order where consecutive threads touch
// consecutive degrees of one (field, sign): fn(j, c, address, imag0).
template <int NT, typename Fn>
__device__ __forceinline__ void for_leaf_block(const CoefIO& io, int m, int p, int j0, int K,
                                               long long c0, Fn&& fn) {
  for (int e = threadIdx.x; e < K * NT; e += 256) {
    const int cc = e & 1;
    const int j = (e >> 1) % K;
    const int c = ((e >> 1) / K) * 2 + cc;
    bool imag0;
    double* a = leaf_ptr(io, m, p, j0, j, c0 + c, imag0);
    fn(j, c, a, imag0);
  }
}

// Staging loop with the global loads of B items per thread issued before any of them is
// used: v = load(e), then put(e, v), for e = threadIdx.x + 256 i < n.
template <typename T, int B = 8, typename Load, typename Put>
__device__ __forceinline__ void staged(int n, Load&& load, Put&& put) {
  for (int e0 = threadIdx.x; e0 < n; e0 += 256 * B) {
    T v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + u * 256;
      if (e < n) v[u] = load(e);
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + u * 256;
      if (e < n) put(e, v[u]);
    }
  }
}

// The K x NT block of a leaf task gathered from the coefficients into xs (row stride LD), in
// the visiting order of for_leaf_block.
template <int NT, int LD>
__device__ __forceinline__ void gather_leaf_block(const CoefIO& io, int m, int p, int j0, int K,
                                                  long long c0, double* xs) {
  staged<double>(
      K * NT,
      [&](int e) {
        const int cc = e & 1;
        const int j = (e >> 1) % K;
        const int c = ((e >> 1) / K) * 2 + cc;
        bool imag0;
        const double* a = leaf_ptr(io, m, p, j0, j, c0 + c, imag0);
        return (a && !imag0) ? *a : 0.0;
      },
      [&](int e, double v) {
        const int cc = e & 1;
        const int j = (e >> 1) % K;
        const int c = ((e >> 1) / K) * 2 + cc;
        xs[j * LD + c] = v;
      });
}

// rows x NT block of an R-wide row buffer (first row `src`) into LDS rows of stride LD.
template <int NT, int LD>
__device__ __forceinline__ void stage_rows(const double* __restrict__ src, int rows, int R, double* dst) {
  staged<double2, 4>(
      rows * (NT / 2),
      [&](int e) {
        const int row = e / (NT / 2), c2 = e % (NT / 2);
        return *reinterpret_cast<const double2*>(src + static_cast<long long>(row) * R + 2 * c2);
      },
      [&](int e, double2 v) {
        const int row = e / (NT / 2), c2 = e % (NT / 2);
        dst[row * LD + 2 * c2] = v.x;
        dst[row * LD + 2 * c2 + 1] = v.y;
      });
}

inline hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

}  // namespace
}  // namespace sht
