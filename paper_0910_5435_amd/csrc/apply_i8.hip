// Butterfly apply in the int8-slice form: every FP64 contraction of the butterfly (levels,
// final skeletons, both directions) runs on the int8 matrix cores (v_mfma_i32_16x16x64_i8),
// FP64 accuracy emulated by fixed-point slices (the Ozaki scheme).
//
// An FP64 operand x is scaled by a power of two shared by its row (factor matrices) or its
// column within the task (vectors), rounded to an integer Z = rint(x 2^(46 - e)) with
// |x| < 2^e, and written as six signed 8-bit digits Z = sum_s d_s 2^(8 (5 - s)).  The low
// digits are two's-complement bytes with their borrow carried upwards, so each digit uses
// all eight bits (d_0 lies in [-65, 65]).  A contraction sum_k a_ik b_kc becomes
//   2^(e_i + e_c - 92) sum_(s,u) 2^(8 (10 - s - u)) sum_k d_s(a_ik) d_u(b_kc),
// and the digit products are exact in the int32 accumulators of the matrix cores.  The
// products with s + u <= kI8Top (21 of 36) are kept, one accumulator per level t = s + u;
// the dropped levels weigh at most 2^-46 of |a|max |b|max per product, about the rounding
// of the 46-bit scaled operands, and the accumulators are turned into FP64 once per
// contraction: y = sum_t acc_t 2^(e_i + e_c - 12 - 8 t).
//
// Factor digits are prepared once per plan (k_i8_prep), tile-packed so one 1 KiB block is
// the A operand of one MFMA for 64 lanes.  Vector digits are cut once per work-group into LDS
// in the B-operand layout: chunk q (64 contraction indices), column tile n (16 columns),
// digit s occupy 1 KiB where lane 16 g + c holds the bytes of indices 64 q + 16 g + t,
// t = 0..15, of column c.  Any assignment of contraction indices to (lane group, byte) works
// as long as A and B use the same one; this one makes every operand a 16-byte access.  The
// 16x16 int32 result sits in the FP32 layout: D[4 (lane / 16) + v][lane % 16] in element v.
//
// Work-groups stage their FP64 vector block in LDS once (coalesced, or gathered from the
// coefficient layout), so the column maxima, the cut and the identity rows never go back to
// global memory, and every wave fetches the A digits of its next (row tile, chunk) unit one
// unit ahead, the first one before the cut, so the factor loads overlap the cut and the
// matrix instructions.
#include <algorithm>
#include <cstdlib>

#include "sht_internal.h"
#include "tile_common.h"

namespace sht {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

static_assert(kI8Dig == 6, "the digit split below produces six digits");
constexpr int kZBits = 46;        // |Z| <= 2^46
constexpr int kDigBlock = 1024;   // bytes of one digit plane of one MFMA operand (64 lanes x 16)
constexpr int kSet = kI8Dig * kDigBlock;  // one (chunk, column tile) of B digits

// The six signed 8-bit digits of Z = rint(x 2^sh) (|Z| <= 2^46), most significant first.
__device__ __forceinline__ void i8_digits(double x, int sh, int (&d)[kI8Dig]) {
  const double z = rint(ldexp(x, sh));
  const double hz = rint(z * 0x1p-24);
  int lo = static_cast<int>(fma(-hz, 0x1p24, z));  // exact: |lo| <= 2^23
  int hi = static_cast<int>(hz);                     // |hi| <= 2^22
  d[5] = ((lo & 255) ^ 128) - 128;
  lo = (lo - d[5]) >> 8;
  d[4] = ((lo & 255) ^ 128) - 128;
  lo = (lo - d[4]) >> 8;
  d[3] = ((lo & 255) ^ 128) - 128;
  hi += (lo - d[3]) >> 8;  // borrow of the low word: 0 or 1
  d[2] = ((hi & 255) ^ 128) - 128;
  hi = (hi - d[2]) >> 8;
  d[1] = ((hi & 255) ^ 128) - 128;
  d[0] = (hi - d[1]) >> 8;
}

// Exponent e with max |x| < 2^e (0 for zero).
__device__ __forceinline__ int exp_of(double m) {
  int e = 0;
  if (m > 0.0) (void)frexp(m, &e);
  return e;
}

struct I8Acc {
  v4i t[kI8Top + 1];
};

__device__ __forceinline__ void i8_zero(I8Acc& a) {
#pragma unroll
  for (int t = 0; t <= kI8Top; ++t) a.t[t] = v4i{0, 0, 0, 0};
}

// One 64-deep chunk: acc_t += sum_(s + u = t) A_s B_u, levels interleaved so consecutive
// matrix instructions write different accumulators.
__device__ __forceinline__ void i8_mma(const v4i (&a)[kI8Dig], const v4i (&b)[kI8Dig], I8Acc& acc) {
#pragma unroll
  for (int r = 0; r < kI8Dig; ++r)
#pragma unroll
    for (int t = r; t <= kI8Top; ++t)
      acc.t[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[r], b[t - r], acc.t[t], 0, 0, 0);
}

// FP64 value of accumulator element v for row exponent er and column exponent ec.
__device__ __forceinline__ double i8_value(const I8Acc& acc, int v, int er, int ec) {
  const int base = er + ec - 12;
  double y = 0.0;
#pragma unroll
  for (int t = kI8Top; t >= 0; --t) y += ldexp(static_cast<double>(acc.t[t][v]), base - 8 * t);
  return y;
}

// A operand of tile m, chunk q (of qk) from the tile-packed digits at `base`.
__device__ __forceinline__ void load_a8(const int8_t* __restrict__ base, long long m, int q, int qk, int lane,
                                        v4i (&a)[kI8Dig]) {
  const v4i* p = reinterpret_cast<const v4i*>(base + ((m * qk + q) * kI8Dig) * kDigBlock) + lane;
#pragma unroll
  for (int s = 0; s < kI8Dig; ++s) a[s] = p[s * 64];
}

// Row exponents of the four rows 16 m + 4 lr + v (v = 0..3) a lane's accumulator elements
// belong to: one 8-byte load (exponent lists are padded to whole 16-row tiles).
__device__ __forceinline__ int4 load_ex4(const int16_t* __restrict__ base, int m, int lr) {
  const int2 w = *reinterpret_cast<const int2*>(base + m * 16 + 4 * lr);
  return make_int4((w.x << 16) >> 16, w.x >> 16, (w.y << 16) >> 16, w.y >> 16);
}
__device__ __forceinline__ int ex_of(const int4& e, int v) { return v == 0 ? e.x : v == 1 ? e.y : v == 2 ? e.z : e.w; }

// B operand of chunk q, column tile n from a digit set in LDS (NTL column tiles).
template <int NTL>
__device__ __forceinline__ void load_b8(const unsigned char* set, int q, int n, int lane, v4i (&b)[kI8Dig]) {
  const v4i* p = reinterpret_cast<const v4i*>(set + (q * NTL + n) * kSet) + lane;
#pragma unroll
  for (int s = 0; s < kI8Dig; ++s) b[s] = p[s * 64];
}

// Column exponents ecol[c] of the n x NT block fetch(j, c); all 256 threads take part.
template <int NT, typename Fetch>
__device__ void i8_col_exps(int n, Fetch&& fetch, double* red, int* ecol) {
  constexpr int G = 256 / NT;
  const int c = threadIdx.x % NT, g = threadIdx.x / NT;
  double mx = 0.0;
  int j = g;
  for (; j + 3 * G < n; j += 4 * G) {  // four independent loads in flight (global sources)
    const double a0 = fetch(j, c), a1 = fetch(j + G, c), a2 = fetch(j + 2 * G, c), a3 = fetch(j + 3 * G, c);
    mx = fmax(mx, fmax(fmax(fabs(a0), fabs(a1)), fmax(fabs(a2), fabs(a3))));
  }
  for (; j < n; j += G) mx = fmax(mx, fabs(fetch(j, c)));
  red[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x < NT) {
    double m = 0.0;
    for (int q = 0; q < G; ++q) m = fmax(m, red[q * NT + threadIdx.x]);
    ecol[threadIdx.x] = exp_of(m);
  }
  __syncthreads();
}

// Digits of the n x NT block fetch(j, c) (zero up to the next multiple of 64) on the column
// grids ecol, written to the digit set `set` in the B layout.  A thread cuts four consecutive
// indices of one column per pass and writes one 32-bit word per digit plane; the 64 threads
// of a wave fill 16 columns x 16 indices, i.e. consecutive words of each plane.
template <int NT, typename Fetch>
__device__ void i8_cut(int n, Fetch&& fetch, const int* ecol, unsigned char* set) {
  constexpr int NTL = NT / 16;
  const int nq = (n + 63) >> 6;
  const int t4 = threadIdx.x & 3, c16 = (threadIdx.x >> 2) & 15, g = threadIdx.x >> 6;
  for (int qn = 0; qn < nq * NTL; ++qn) {
    const int q = qn / NTL, nt = qn % NTL;
    const int c = nt * 16 + c16;
    const int j0 = 64 * q + 16 * g + 4 * t4;
    const int sh = kZBits - ecol[c];
    unsigned w[kI8Dig];
#pragma unroll
    for (int s = 0; s < kI8Dig; ++s) w[s] = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (j0 + u < n) {
        int d[kI8Dig];
        i8_digits(fetch(j0 + u, c), sh, d);
#pragma unroll
        for (int s = 0; s < kI8Dig; ++s) w[s] |= static_cast<unsigned>(d[s] & 255) << (8 * u);
      }
    }
    unsigned* dst = reinterpret_cast<unsigned*>(set + qn * kSet) + (16 * g + c16) * 4 + t4;
#pragma unroll
    for (int s = 0; s < kI8Dig; ++s) dst[s * (kDigBlock / 4)] = w[s];
  }
}

// ------------------------------------------------------------------ factor digit preparation
// One stored matrix M (rows x cols, column-major at fac + off) per work-group, both
// orientations: A = M (o = 0) and A = M^T (o = 1), row exponents then tile-packed digits.
__global__ void __launch_bounds__(256) k_i8_prep(const double* __restrict__ fac, const I8Block* __restrict__ blocks,
                                                 int8_t* __restrict__ dig, int16_t* __restrict__ dex) {
  __shared__ int ex_s[4096];
  const I8Block b = blocks[blockIdx.x];
  for (int o = 0; o < 2; ++o) {
    const int ar = o ? b.cols : b.rows, ak = o ? b.rows : b.cols;
    const int tm = (ar + 15) / 16, qk = (ak + 63) / 64;
    auto A = [&](int i, int k) {
      return o ? fac[b.off + k + static_cast<long long>(i) * b.rows] : fac[b.off + i + static_cast<long long>(k) * b.rows];
    };
    __syncthreads();
    for (int i = threadIdx.x; i < tm * 16; i += 256) {
      double mx = 0.0;
      if (i < ar)
        for (int k = 0; k < ak; ++k) mx = fmax(mx, fabs(A(i, k)));
      const int e = exp_of(mx);
      ex_s[i] = e;
      dex[b.o.ex[o] + i] = static_cast<int16_t>(e);
    }
    __syncthreads();
    unsigned* base = reinterpret_cast<unsigned*>(dig + b.o.dig[o]);
    const long long units = static_cast<long long>(tm) * qk * 256;
    for (long long u = threadIdx.x; u < units; u += 256) {
      const int t4 = static_cast<int>(u & 3), L = static_cast<int>((u >> 2) & 63);
      const long long mq = u >> 8;
      const int i = static_cast<int>(mq / qk) * 16 + (L & 15);
      const int k0 = static_cast<int>(mq % qk) * 64 + 16 * (L >> 4) + 4 * t4;
      const int sh = kZBits - ex_s[i];
      unsigned w[kI8Dig] = {};
      for (int j = 0; j < 4; ++j) {
        if (i < ar && k0 + j < ak) {
          int d[kI8Dig];
          i8_digits(A(i, k0 + j), sh, d);
          for (int s = 0; s < kI8Dig; ++s) w[s] |= static_cast<unsigned>(d[s] & 255) << (8 * j);
        }
      }
      unsigned* dst = base + mq * (kSet / 4) + L * 4 + t4;
      for (int s = 0; s < kI8Dig; ++s) dst[s * (kDigBlock / 4)] = w[s];
    }
  }
}

// The outputs of a level task are taken one at a time: the digits of the output's contraction
// operand are cut into LDS, then its row tiles are dealt to the four waves, each walking its
// (tile, chunk) units in order and loading the A digits of the next unit (continuing into the
// next output) before the matrix instructions of the current one.  The first unit's loads are
// issued before the first cut.

// ------------------------------------------------------------------- level, synthesis
// out_o = in[skel_o] + T_o in[red_o].  LDS: the K x (NT + 2) FP64 input block, the digit set of
// the current output (its red rows, in red order; setb bytes), then the index lists
// [skel0 red0 skel1 red1].
template <int NT>
__global__ void __launch_bounds__(256, 2)
k_level_synth_i8(const LevelTask* __restrict__ tasks, long long ntasks, int nblk, const int8_t* __restrict__ dig,
                 const int16_t* __restrict__ dex, const uint16_t* __restrict__ idx,
                 const PairDesc* __restrict__ pairs, const double* __restrict__ in, double* __restrict__ out, int R,
                 CoefIO io, int setb) {
  extern __shared__ __align__(16) unsigned char lds8[];
  __shared__ double red_s[256];
  __shared__ int ecol[NT];
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const LevelTask& tk = tasks[ti];  // (a reference: per-output fields are picked at run time)
  const int K = tk.K;
  const int nouts = tk.k[1] < 0 ? 1 : 2;
  const int k0 = tk.k[0], k1 = nouts > 1 ? tk.k[1] : 0;
  const long long c0 = static_cast<long long>(blk) * NT;
  double* xs = reinterpret_cast<double*>(lds8);
  unsigned char* set = lds8 + static_cast<size_t>(K) * LD * 8;
  uint16_t* ix = reinterpret_cast<uint16_t*>(set + setb);
  for (int o = 0; o < nouts; ++o)
    for (int e = threadIdx.x; e < K; e += 256) ix[o * K + e] = idx[tk.idx[o] + e];
  if (io.on() && tk.mp >= 0) {
    const PairDesc pd = pairs[tk.mp];
    gather_leaf_block<NT, LD>(io, pd.m, pd.p, tk.in_row - pd.in_base, K, c0, xs);
  } else {
    stage_rows<NT, LD>(in + static_cast<long long>(tk.in_row) * R + c0, K, R, xs);
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lc = lane & 15, lr = lane >> 4;
  const int nm[2] = {(k0 + 15) >> 4, (k1 + 15) >> 4};
  const int nqs[2] = {(K - k0 + 63) >> 6, (K - k1 + 63) >> 6};
  // a unit's A digits; with the tile's first chunk also its row exponents
  auto load_unit = [&](int o, int mt, int q, v4i (&a)[kI8Dig], int4& e) {
    if (q < nqs[o]) {
      load_a8(dig + (o ? tk.i8[1].dig[0] : tk.i8[0].dig[0]), mt, q, nqs[o], lane, a);
      if (q == 0) e = load_ex4(dex + (o ? tk.i8[1].ex[0] : tk.i8[0].ex[0]), mt, lr);
    }
  };
  v4i an[kI8Dig];
  int4 en = make_int4(0, 0, 0, 0), et = en;
  if (wave < nm[0]) load_unit(0, wave, 0, an, en);
  else if (nouts > 1 && wave < nm[1]) load_unit(1, wave, 0, an, en);
  __syncthreads();
  i8_col_exps<NT>(K, [&](int j, int c) { return xs[j * LD + c]; }, red_s, ecol);  // (also publishes ix)
  int ec[NTL];
#pragma unroll
  for (int n = 0; n < NTL; ++n) ec[n] = ecol[n * 16 + lc];
  for (int o = 0; o < nouts; ++o) {
    const int k = o ? k1 : k0;
    const uint16_t* red = ix + o * K + k;
    if (o) __syncthreads();  // the previous output's units are done with the digit set
    i8_cut<NT>(K - k, [&](int j, int c) { return xs[static_cast<int>(red[j]) * LD + c]; }, ecol, set);
    __syncthreads();
    const int nq = nqs[o];
    const uint16_t* skel = ix + o * K;
    double* ob = out + static_cast<long long>(o ? tk.out_row[1] : tk.out_row[0]) * R + c0;
    I8Acc acc[NTL];
    for (int mt = wave, q = 0; mt < nm[o];) {
      v4i a[kI8Dig];
#pragma unroll
      for (int s = 0; s < kI8Dig; ++s) a[s] = an[s];
      int mt2 = mt, q2 = q + 1;
      if (q2 >= nq) {
        mt2 = mt + 4;
        q2 = 0;
      }
      if (q == 0) et = en;
      if (mt2 < nm[o]) load_unit(o, mt2, q2, an, en);
      else if (o + 1 < nouts && wave < nm[1]) load_unit(1, wave, 0, an, en);  // the next output's first unit
      if (q == 0) {
#pragma unroll
        for (int n = 0; n < NTL; ++n) i8_zero(acc[n]);
      }
      if (q < nq) {
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          v4i b[kI8Dig];
          load_b8<NTL>(set, q, n, lane, b);
          i8_mma(a, b, acc[n]);
        }
      }
      if (q2 == 0) {  // last chunk of this tile: out rows = identity rows + contraction
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = mt * 16 + 4 * lr + v;
          if (row < k) {
            const int erow = ex_of(et, v);
            const double* xr = xs + static_cast<int>(skel[row]) * LD;
#pragma unroll
            for (int n = 0; n < NTL; ++n) {
              const int col = n * 16 + lc;
              ob[static_cast<long long>(row) * R + col] = xr[col] + i8_value(acc[n], v, erow, ec[n]);
            }
          }
        }
      }
      mt = mt2;
      q = q2;
    }
  }
}

// ------------------------------------------------------------------ level, transposed
// in = sum_o (w_o at rows skel_o) + (T_o^T w_o at rows red_o) into an FP64 block in LDS, one
// output at a time: every row gets exactly one term from each output, so output 0 stores its
// terms and output 1 adds its own, with no clearing and no atomics.  LDS: the K x (NT + 2) FP64
// block, the current output's w_o staged with batched loads (max(k_0, k_1) x (NT + 2) FP64),
// its digit set (setb bytes), then the index lists.
template <int NT>
__global__ void __launch_bounds__(256, 2)
k_level_trans_i8(const LevelTask* __restrict__ tasks, long long ntasks, int nblk, const int8_t* __restrict__ dig,
                 const int16_t* __restrict__ dex, const uint16_t* __restrict__ idx,
                 const PairDesc* __restrict__ pairs, const double* __restrict__ win, double* __restrict__ xout,
                 int R, CoefIO io, int setb) {
  extern __shared__ __align__(16) unsigned char lds8[];
  __shared__ double red_s[256];
  __shared__ int ecol[NT];
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const LevelTask& tk = tasks[ti];
  const int K = tk.K;
  const int nouts = tk.k[1] < 0 ? 1 : 2;
  const int k0 = tk.k[0], k1 = nouts > 1 ? tk.k[1] : 0;
  const long long c0 = static_cast<long long>(blk) * NT;
  double* acc_l = reinterpret_cast<double*>(lds8);
  double* wl = acc_l + K * LD;  // the current output's w_o (k_o rows)
  unsigned char* set = reinterpret_cast<unsigned char*>(wl + (k0 > k1 ? k0 : k1) * LD);
  uint16_t* ix = reinterpret_cast<uint16_t*>(set + setb);
  for (int o = 0; o < nouts; ++o)
    for (int e = threadIdx.x; e < K; e += 256) ix[o * K + e] = idx[tk.idx[o] + e];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lc = lane & 15, lr = lane >> 4;
  const int nm[2] = {(K - k0 + 15) >> 4, nouts > 1 ? (K - k1 + 15) >> 4 : 0};
  const int nqs[2] = {(k0 + 63) >> 6, (k1 + 63) >> 6};
  auto load_unit = [&](int o, int mt, int q, v4i (&a)[kI8Dig], int4& e) {
    if (q < nqs[o]) {
      load_a8(dig + (o ? tk.i8[1].dig[1] : tk.i8[0].dig[1]), mt, q, nqs[o], lane, a);
      if (q == 0) e = load_ex4(dex + (o ? tk.i8[1].ex[1] : tk.i8[0].ex[1]), mt, lr);
    }
  };
  v4i an[kI8Dig];
  int4 en = make_int4(0, 0, 0, 0), et = en;
  if (wave < nm[0]) load_unit(0, wave, 0, an, en);
  else if (wave < nm[1]) load_unit(1, wave, 0, an, en);
  for (int o = 0; o < nouts; ++o) {
    const int k = o ? k1 : k0;
    // w_o into LDS with batched loads (the output-0 units never read this region)
    stage_rows<NT, LD>(win + static_cast<long long>(o ? tk.out_row[1] : tk.out_row[0]) * R + c0, k, R, wl);
    __syncthreads();  // (also publishes ix, and ends output 0's units)
    auto fw = [&](int j, int c) { return wl[j * LD + c]; };
    i8_col_exps<NT>(k, fw, red_s, ecol);
    i8_cut<NT>(k, fw, ecol, set);
    // identity part: w_o at the skeleton rows (output 0 stores, output 1 adds)
    const uint16_t* skel = ix + o * K;
    for (int e = threadIdx.x; e < k * NT; e += 256) {
      double* d = acc_l + static_cast<int>(skel[e / NT]) * LD + e % NT;
      const double val = wl[(e / NT) * LD + e % NT];
      *d = o ? *d + val : val;
    }
    __syncthreads();
    const int nq = nqs[o];
    const int nr = K - k;
    const uint16_t* red = ix + o * K + k;
    int ec[NTL];
#pragma unroll
    for (int n = 0; n < NTL; ++n) ec[n] = ecol[n * 16 + lc];
    I8Acc acc[NTL];
    for (int mt = wave, q = 0; mt < nm[o];) {
      v4i a[kI8Dig];
#pragma unroll
      for (int s = 0; s < kI8Dig; ++s) a[s] = an[s];
      int mt2 = mt, q2 = q + 1;
      if (q2 >= nq) {
        mt2 = mt + 4;
        q2 = 0;
      }
      if (q == 0) et = en;
      if (mt2 < nm[o]) load_unit(o, mt2, q2, an, en);
      else if (o + 1 < nouts && wave < nm[1]) load_unit(1, wave, 0, an, en);
      if (q == 0) {
#pragma unroll
        for (int n = 0; n < NTL; ++n) i8_zero(acc[n]);
      }
      if (q < nq) {
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          v4i b[kI8Dig];
          load_b8<NTL>(set, q, n, lane, b);
          i8_mma(a, b, acc[n]);
        }
      }
      if (q2 == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = mt * 16 + 4 * lr + v;
          if (j < nr) {
            const int ej = ex_of(et, v);
            double* dst = acc_l + static_cast<int>(red[j]) * LD;
#pragma unroll
            for (int n = 0; n < NTL; ++n) {
              const double val = i8_value(acc[n], v, ej, ec[n]);
              dst[n * 16 + lc] = o ? dst[n * 16 + lc] + val : val;
            }
          }
        }
      }
      mt = mt2;
      q = q2;
    }
  }
  __syncthreads();
  if (io.on() && tk.mp >= 0) {
    const PairDesc pd = pairs[tk.mp];
    for_leaf_block<NT>(io, pd.m, pd.p, tk.in_row - pd.in_base, K, c0, [&](int j, int c, double* a, bool imag0) {
      if (a) *a = imag0 ? 0.0 : acc_l[j * LD + c];
    });
    return;
  }
  double* xb = xout + static_cast<long long>(tk.in_row) * R + c0;
  for (int e = threadIdx.x; e < K * (NT / 2); e += 256) {
    const int row = e / (NT / 2), c2 = e % (NT / 2);
    *reinterpret_cast<double2*>(xb + static_cast<long long>(row) * R + 2 * c2) =
        make_double2(acc_l[row * LD + 2 * c2], acc_l[row * LD + 2 * c2 + 1]);
  }
}

// ------------------------------------------------------------------- final, synthesis
// E = S_0 v_0, O = S_1 v_1 per 16-row tile; g(+-x) = (E +- O) / D.  LDS: the digit sets of v_0
// and v_1 (setb bytes each; v_p is read from global memory twice, the second time from
// cache).  A wave's units are (tile, parity, chunk); E and O of a tile are combined after its
// last unit.
template <int NT>
__global__ void __launch_bounds__(256, 2)
k_final_synth_i8(const FinalTask* __restrict__ tasks, long long ntasks, int nblk, const int8_t* __restrict__ dig,
                 const int16_t* __restrict__ dex, const double* __restrict__ v0buf, const double* __restrict__ v1buf,
                 const double* __restrict__ invD, double* __restrict__ Y, int l, int R, int setb) {
  extern __shared__ __align__(16) unsigned char lds8[];
  __shared__ double red_s[256];
  __shared__ int ecol[2][NT];
  constexpr int NTL = NT / 16;
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const FinalTask& ft = tasks[ti];
  const long long c0 = static_cast<long long>(blk) * NT;
  const double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1];
  const int h = ft.h;
  unsigned char* sets = lds8;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lc = lane & 15, lr = lane >> 4;
  const int nq0 = (k0 + 63) >> 6, nq1 = (k1 + 63) >> 6;
  const int nu = nq0 + nq1;  // units per tile: parity 0 chunks, then parity 1 chunks
  const int nm = (h + 15) >> 4;
  // a unit's A digits; with a tile's first unit also the row exponents of both parities
  auto load_unit = [&](int mt, int u, v4i (&a)[kI8Dig], int4& e0, int4& e1) {
    if (u == 0) {
      if (k0 > 0) e0 = load_ex4(dex + ft.i8[0].ex[0], mt, lr);
      if (k1 > 0) e1 = load_ex4(dex + ft.i8[1].ex[0], mt, lr);
    }
    if (u < nq0) load_a8(dig + ft.i8[0].dig[0], mt, u, nq0, lane, a);
    else if (u < nu) load_a8(dig + ft.i8[1].dig[0], mt, u - nq0, nq1, lane, a);
  };
  v4i an[kI8Dig];
  int4 en0 = make_int4(0, 0, 0, 0), en1 = en0, et0 = en0, et1 = en0;
  if (wave < nm) load_unit(wave, 0, an, en0, en1);
  for (int p = 0; p < 2; ++p) {
    const double* v = V + static_cast<long long>(p ? ft.in_row[1] : ft.in_row[0]) * R + c0;
    auto fv = [&](int j, int c) { return v[static_cast<long long>(j) * R + c]; };
    i8_col_exps<NT>(p ? k1 : k0, fv, red_s, ecol[p]);
    i8_cut<NT>(p ? k1 : k0, fv, ecol[p], sets + p * setb);
  }
  __syncthreads();
  I8Acc acc[2][NTL];
  for (int mt = wave, u = 0; mt < nm;) {
    v4i a[kI8Dig];
#pragma unroll
    for (int s = 0; s < kI8Dig; ++s) a[s] = an[s];
    int mt2 = mt, u2 = u + 1;
    if (u2 >= nu) {
      mt2 = mt + 4;
      u2 = 0;
    }
    if (u == 0) {
      et0 = en0;
      et1 = en1;
    }
    if (mt2 < nm) load_unit(mt2, u2, an, en0, en1);
    if (u == 0) {
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        i8_zero(acc[0][n]);
        i8_zero(acc[1][n]);
      }
    }
    if (u < nq0) {
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        v4i b[kI8Dig];
        load_b8<NTL>(sets, u, n, lane, b);
        i8_mma(a, b, acc[0][n]);
      }
    } else if (u < nu) {
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        v4i b[kI8Dig];
        load_b8<NTL>(sets + setb, u - nq0, n, lane, b);
        i8_mma(a, b, acc[1][n]);
      }
    }
    if (u2 == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = mt * 16 + 4 * lr + v;
        if (ii < h) {
          const int row = ft.row0 + ii;
          const double sc = invD[row];
          const int e0 = ex_of(et0, v), e1 = ex_of(et1, v);
          double* yp = Y + y_row(l, ft.m, l + row) * R + c0;
          double* ym = Y + y_row(l, ft.m, l - 1 - row) * R + c0;
#pragma unroll
          for (int n = 0; n < NTL; ++n) {
            const int col = n * 16 + lc;
            const double e = i8_value(acc[0][n], v, e0, ecol[0][col]);
            const double od = i8_value(acc[1][n], v, e1, ecol[1][col]);
            yp[col] = (e + od) * sc;
            ym[col] = (e - od) * sc;
          }
        }
      }
    }
    mt = mt2;
    u = u2;
  }
}

// ------------------------------------------------------------------ final, transposed
// v_p = S_p^T (half scale (G(+x) +- G(-x))) over row chunks of ICH: each chunk's folded rows
// get their own column grids, so the int32 sums of a chunk are added into FP64 sums kept in
// LDS (one row per output row of both parities, each row tile owned by one wave).  LDS: the
// (k_0 + k_1) x NT FP64 sums (accb bytes), the folded chunk (2 x ICH x (NT + 2) FP64), then the
// digit sets of its two parities.
template <int NT, int ICH>
__global__ void __launch_bounds__(256, 2)
k_final_trans_i8(const FinalTask* __restrict__ tasks, long long ntasks, int nblk, const int8_t* __restrict__ dig,
                 const int16_t* __restrict__ dex, const double* __restrict__ Yin, const double* __restrict__ scale,
                 double half, double* __restrict__ v0buf, double* __restrict__ v1buf, int l, int R, int accb,
                 int setb) {
  extern __shared__ __align__(16) unsigned char lds8[];
  __shared__ double red_s[256];
  __shared__ int ecol[2][NT];
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  static_assert(ICH % 64 == 0, "chunks of whole 64-row digit blocks");
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const FinalTask& ft = tasks[ti];
  const long long c0 = static_cast<long long>(blk) * NT;
  double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1];
  const int h = ft.h;
  const int qh = (h + 63) >> 6;  // contraction chunks of S_p^T
  double* sums = reinterpret_cast<double*>(lds8);  // rows [0, k0): parity 0, [k0, k0 + k1): parity 1
  double* eo = reinterpret_cast<double*>(lds8 + accb);  // folded chunk: E rows, then O rows
  unsigned char* sets = reinterpret_cast<unsigned char*>(eo + 2 * ICH * LD);
  for (int e = threadIdx.x; e < (k0 + k1) * NT; e += 256) sums[e] = 0.0;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lc = lane & 15, lr = lane >> 4;
  const int nm0 = (k0 + 15) >> 4, ntot = nm0 + ((k1 + 15) >> 4);
  auto load_unit = [&](int tq, int cq, v4i (&a)[kI8Dig], int4& e) {
    const int p = tq < nm0 ? 0 : 1;
    load_a8(dig + (p ? ft.i8[1].dig[1] : ft.i8[0].dig[1]), p ? tq - nm0 : tq, cq, qh, lane, a);
    e = load_ex4(dex + (p ? ft.i8[1].ex[1] : ft.i8[0].ex[1]), p ? tq - nm0 : tq, lr);
  };
  for (int i0 = 0; i0 < h; i0 += ICH) {
    const int ih = min(ICH, h - i0);
    const int nq = (ih + 63) >> 6;
    v4i an[kI8Dig];
    int4 en = make_int4(0, 0, 0, 0), et = en;
    if (wave < ntot) load_unit(wave, i0 / 64, an, en);
    __syncthreads();
    staged<double2, 2>(
        ih * NT,
        [&](int e) {
          const int row = ft.row0 + i0 + e / NT, c = e % NT;
          return make_double2(Yin[y_row(l, ft.m, l + row) * R + c0 + c], Yin[y_row(l, ft.m, l - 1 - row) * R + c0 + c]);
        },
        [&](int e, double2 g) {
          const int i = e / NT, c = e % NT;
          const double sc = half * scale[ft.row0 + i0 + i];
          eo[i * LD + c] = (g.x + g.y) * sc;
          eo[(ICH + i) * LD + c] = (g.x - g.y) * sc;
        });
    __syncthreads();
    for (int p = 0; p < 2; ++p) {
      const double* src = eo + (p ? ICH : 0) * LD;
      auto fs = [&](int j, int c) { return src[j * LD + c]; };
      i8_col_exps<NT>(ih, fs, red_s, ecol[p]);
      i8_cut<NT>(ih, fs, ecol[p], sets + p * setb);
    }
    __syncthreads();
    I8Acc acc[NTL];
    for (int tq = wave, cq = 0; tq < ntot;) {
      const int p = tq < nm0 ? 0 : 1;
      const int mt = p ? tq - nm0 : tq;
      v4i a[kI8Dig];
#pragma unroll
      for (int s = 0; s < kI8Dig; ++s) a[s] = an[s];
      int tq2 = tq, cq2 = cq + 1;
      if (cq2 >= nq) {
        tq2 = tq + 4;
        cq2 = 0;
      }
      if (cq == 0) et = en;
      if (tq2 < ntot) load_unit(tq2, i0 / 64 + cq2, an, en);
      if (cq == 0) {
#pragma unroll
        for (int n = 0; n < NTL; ++n) i8_zero(acc[n]);
      }
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        v4i b[kI8Dig];
        load_b8<NTL>(sets + p * setb, cq, n, lane, b);
        i8_mma(a, b, acc[n]);
      }
      if (cq2 == 0) {
        const int kp = p ? k1 : k0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a_ = mt * 16 + 4 * lr + v;
          if (a_ < kp) {
            double* srow = sums + (p ? k0 + a_ : a_) * NT;
#pragma unroll
            for (int n = 0; n < NTL; ++n)
              srow[n * 16 + lc] += i8_value(acc[n], v, ex_of(et, v), ecol[p][n * 16 + lc]);
          }
        }
      }
      tq = tq2;
      cq = cq2;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < (k0 + k1) * NT; e += 256) {
    const int r = e / NT, c = e % NT;
    const bool odd = r >= k0;
    const int a = odd ? r - k0 : r;
    V[static_cast<long long>((odd ? ft.in_row[1] : ft.in_row[0]) + a) * R + c0 + c] = sums[e];
  }
}

// LDS bytes of one digit set: ceil(n / 64) chunks x NT / 16 column tiles.
long long set_bytes(int n, int nt) { return static_cast<long long>((n + 63) / 64) * (nt / 16) * kSet; }

constexpr long long kLdsMax = 150 * 1024;  // dynamic LDS one work-group may take
constexpr long long kLds2 = 76 * 1024;     // two work-groups per compute unit

// Widest column tile (32 or 16, dividing R) whose LDS `need(nt)` allows two work-groups per
// CU, else the widest that fits at all; 0 if none does.  (64 columns would take two row tiles x
// four column tiles x five int32 accumulators per wave: more registers than two waves per SIMD
// leave.)
template <typename Need>
int pick_nt(int R, Need&& need) {
  for (int nt : {32, 16})
    if (R % nt == 0 && need(nt) <= kLds2) return nt;
  for (int nt : {32, 16})
    if (R % nt == 0 && need(nt) <= kLdsMax) return nt;
  return 0;
}

#define I8_PICK(NT_, KER, ...)                                                              \
  do {                                                                                      \
    if ((e = allow_lds(reinterpret_cast<const void*>(&KER<NT_>), lds)) != hipSuccess) return e; \
    hipLaunchKernelGGL(KER<NT_>, grid, dim3(256), lds, s, __VA_ARGS__);                     \
  } while (0)

}  // namespace

hipError_t i8_prepare(sht_plan_s* P, hipStream_t s) {
  if (P->d.dig) return hipSuccess;
  if (!P->d.fac || !P->d.i8blocks) return hipErrorInvalidValue;
  // k_i8_prep keeps one exponent per row of an operand in LDS: at most 4096 rows (finals have
  // at most l <= 2048 rows, level blocks at most K)
  for (int K : P->step_maxK)
    if (K > 4096) return hipErrorInvalidValue;
  if (P->final_maxh > 4096) return hipErrorInvalidValue;
  int8_t* dig = nullptr;
  int16_t* dex = nullptr;
  hipError_t e = dev_alloc(reinterpret_cast<void**>(&dig), std::max<long long>(P->n_dig, 1024));
  if (e == hipSuccess) e = dev_alloc(reinterpret_cast<void**>(&dex), std::max<long long>(P->n_dex, 16) * sizeof(int16_t));
  for (long long b0 = 0; e == hipSuccess && b0 < P->n_blocks; b0 += 1 << 20) {
    const long long nb = std::min<long long>(1 << 20, P->n_blocks - b0);
    hipLaunchKernelGGL(k_i8_prep, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, P->d.fac, P->d.i8blocks + b0,
                       dig, dex);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    if (dig) (void)hipFree(dig);
    if (dex) (void)hipFree(dex);
    return e;
  }
  P->d.dig = dig;
  P->d.dex = dex;
  P->stats.device_bytes += P->n_dig + 2 * P->n_dex;
  return hipSuccess;
}

hipError_t launch_level_i8(const sht_plan_s* P, int step, bool transpose, const double* in, double* out, int R,
                           hipStream_t s, double* coeff, int only) {
  const CoefIO io{coeff, nullptr, P->kind == SHT_COMPLEX ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l, P->l,
                  P->kind};
  for (size_t c = 0; c < P->step_classes[step].size(); ++c) {
    if (only >= 0 && static_cast<int>(c) != only) continue;
    const LaunchClass& lc = P->step_classes[step][c];
    const long long cnt = lc.cnt;
    if (cnt == 0) continue;
    const LevelTask* tasks = P->d.tasks + P->step_off[step] + lc.off;
    const int K = lc.maxK;
    // contraction length per output: synthesis K - k (red rows), transposed k (w rows)
    const int kd = transpose ? lc.maxk : lc.maxnr;
    // FP64 block of K rows (the staged input, or the transposed sums plus one staged output
    // vector), one digit set, indices
    const long long rows = transpose ? static_cast<long long>(K) + lc.maxk : K;
    auto need = [&](int nt) { return set_bytes(kd, nt) + 4LL * K + rows * (nt + 2) * 8; };
    const int NT = pick_nt(R, need);
    if (NT == 0) return hipErrorInvalidConfiguration;
    const int setb = static_cast<int>(set_bytes(kd, NT));
    const size_t lds = static_cast<size_t>(need(NT));
    const int nblk = R / NT;
    const dim3 grid(xcd_grid(cnt, nblk));
    hipError_t e;
    if (!transpose) {
      if (NT == 32) I8_PICK(32, k_level_synth_i8, tasks, cnt, nblk, P->d.dig, P->d.dex, P->d.idx, P->d.pairs, in, out, R, io, setb);
      else I8_PICK(16, k_level_synth_i8, tasks, cnt, nblk, P->d.dig, P->d.dex, P->d.idx, P->d.pairs, in, out, R, io, setb);
    } else {
      if (NT == 32) I8_PICK(32, k_level_trans_i8, tasks, cnt, nblk, P->d.dig, P->d.dex, P->d.idx, P->d.pairs, in, out, R, io, setb);
      else I8_PICK(16, k_level_trans_i8, tasks, cnt, nblk, P->d.dig, P->d.dex, P->d.idx, P->d.pairs, in, out, R, io, setb);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_final_i8(const sht_plan_s* P, bool transpose, const double* v0, const double* v1, double* v0w,
                           double* v1w, double* y, const double* yin, int R, bool adjoint, hipStream_t s, int only) {
  hipError_t e;
  if (!transpose) {
    for (size_t c = 0; c < P->final_classes.size(); ++c) {
      if (only >= 0 && static_cast<int>(c) != only) continue;
      const LaunchClass& lc = P->final_classes[c];
      const long long cnt = lc.cnt;
      if (cnt == 0) continue;
      const FinalTask* tasks = P->d.finals + lc.off;
      auto need = [&](int nt) { return 2 * set_bytes(lc.maxk, nt); };
      const int NT = pick_nt(R, need);
      if (NT == 0) return hipErrorInvalidConfiguration;
      const int setb = static_cast<int>(set_bytes(lc.maxk, NT));
      const size_t lds = static_cast<size_t>(need(NT));
      const int nblk = R / NT;
      const dim3 grid(xcd_grid(cnt, nblk));
      if (NT == 32) I8_PICK(32, k_final_synth_i8, tasks, cnt, nblk, P->d.dig, P->d.dex, v0, v1, P->d.invD, y, P->l, R, setb);
      else I8_PICK(16, k_final_synth_i8, tasks, cnt, nblk, P->d.dig, P->d.dex, v0, v1, P->d.invD, y, P->l, R, setb);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  constexpr int ICH = 64;
  const long long cnt = P->n_final;
  const double* scale = adjoint ? P->d.invD : P->d.D;
  const double half = adjoint ? 1.0 : 0.5;
  // 16 columns: the FP64 sums of both parities' rows stay in LDS across the row chunks
  constexpr int NT = 16;
  const int setb = static_cast<int>(set_bytes(ICH, NT));
  const int accb = 2 * P->final_maxk * NT * 8;
  const size_t lds = static_cast<size_t>(accb) + 2 * ICH * (NT + 2) * 8 + 2 * static_cast<size_t>(setb);
  if (static_cast<long long>(lds) > kLdsMax) return hipErrorInvalidConfiguration;
  const int nblk = R / NT;
  const dim3 grid(xcd_grid(cnt, nblk));
  if ((e = allow_lds(reinterpret_cast<const void*>(&k_final_trans_i8<NT, ICH>), lds)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_final_trans_i8<NT, ICH>), grid, dim3(256), lds, s, P->d.finals, cnt, nblk, P->d.dig, P->d.dex,
                     yin, scale, half, v0w, v1w, P->l, R, accb, setb);
  return hipGetLastError();
}

}  // namespace sht
