// Butterfly apply on the matrix cores, used when the number of R columns is a multiple of
// 16, i.e. many fields at once.  Three arithmetic variants share the kernels:
//
//  * FP64: v_mfma_f64_16x16x4f64.
//  * split: every FP64 operand x is cut into x1 + x2 where x1 keeps the top bits on a grid
//    common to its row (factors) or column (vectors), |x1| <= 2^11 grid units, and x2 =
//    fp32(x - x1).  One K-step sums four products a1 b1 of at most 2^22 grid units each,
//    which FP32 holds exactly (2^24), so it runs on v_mfma_f32_16x16x4f32 without rounding
//    and is added into an FP64 accumulator after every K-step; the correction products
//    a2 b2 + a2 b1 + a1 b2 (about 2^-22 and 2^-11 of the result, chained smallest first)
//    are summed in FP32 for one K-step and then added into the FP64 accumulator as well,
//    which keeps their rounding near 2^-35 of the result.  Factor slices are prepared once
//    per plan; vector slices are cut on the fly from per-task, per-column scales.
//  * FP32: plain v_mfma_f32_16x16x4f32 on the FP32 sum of a factor's split pair and on
//    fp32(b), FP32 accumulation.
//
// Each interpolation is a small GEMM with a gathered operand: out = in[skel] + T in[red]
// (synthesis) or in = sum_o scatter(T_o^T w_o, w_o) (transposed).  A work-group takes one
// task and NT columns; every wave runs pairs of 16-row tiles with the factor fragments (A)
// fetched kPrefetch K-steps ahead from global memory (a stored column is contiguous, so 16 lanes
// read consecutive words) and the vector fragments (B) from LDS or global memory.
// Work-groups are numbered so that all column blocks of one task land on the same XCD
// (ids are dealt round-robin over the 8 XCDs): the factor block is read from HBM once and
// served to the other column blocks from that XCD's L2.
//
// Register layouts (checked on gfx950): for both 16x16x4 shapes A[i][k] sits in lane
// i + 16k and B[k][j] in lane j + 16k; the FP64 result D[4v + lane/16][lane%16] is in
// element v, the FP32 result D[4(lane/16) + v][lane%16].  With NT = 16 NTL columns per
// work-group, column tile n of a lane with lane%16 = c is work-group column c NTL + n: a
// lane's columns are adjacent, so its B entries and results of one row move as one 16-byte
// access.
#include <algorithm>
#include <cstdlib>

#include "sht_internal.h"
#include "tile_common.h"

namespace sht {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kSliceBits = 11;  // |x1| <= 2^11 units of the row / column grid
constexpr int kPrefetch = 4;    // K-steps of factor fragments fetched ahead (double-buffered)
// Work-groups per compute unit the apply kernels are compiled for: two keep two waves on
// every SIMD (at most 256 registers per lane), so one wave's stalls are covered by another
// (three made no difference where they fit without spilling).
constexpr int kMinBlocks = 2;

enum { P64 = 0, PSPLIT = 1, P32 = 2 };

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of the 16x16 tile held in accumulator element v of a lane with lane/16 = lr.
template <int PREC>
__device__ __forceinline__ int drow(int v, int lr) { return PREC == P64 ? 4 * v + lr : 4 * lr + v; }

// ---------------------------------------------------------------- operands and accumulators

template <int PREC> struct AFrag;
template <> struct AFrag<P64> { double a; };
template <> struct AFrag<PSPLIT> { float a1, a2; };
template <> struct AFrag<P32> { float a1, a2; };  // summed at the MFMA, after the load lands

// FP32 fragment loads are branch-free: the load always happens (from `safe`, an entry of the
// same block, where ok is false) and the zero is selected afterwards, because a per-lane
// condition around a load compiles to a divergent branch per K-step, which costs more than
// the cheap FP32 MFMA it guards.  For FP64 and split FP32 the MFMA work per step is larger
// and skipping the masked loads measured faster.
template <int PREC> constexpr bool kBranchFree = PREC == P32;

// Which K loop a level kernel compiles for a wave's row tiles: 0 a lone tile, 1 a pair, 2 one
// loop that tests at run time whether the second tile exists.
template <int V>
struct TileCount {
  static constexpr int value = V;
};

// Entry p[i] where ok holds, else 0 (branch-free for the precisions that ask for it).
template <int PREC, class T>
__device__ __forceinline__ T sel_load(const T* p, long long i, bool ok, long long safe) {
  if constexpr (kBranchFree<PREC>) {
    const T v = p[ok ? i : safe];
    return ok ? v : T(0);
  } else {
    return ok ? p[i] : T(0);
  }
}

// Factor fragment entry i where ok holds.  Split and FP32: where it does not, the entry at
// `safe` (the block's first) is loaded instead and used as it is: such a fragment either
// meets zero B entries (past the end of the contraction) or feeds output rows that are
// never stored, and every stored factor is finite, so it contributes nothing.  Loading
// unconditionally and not touching the value until the MFMA keeps the prefetched loads in
// flight.  FP64 skips the masked loads and substitutes 0, which measured slightly faster.
template <int PREC>
__device__ __forceinline__ AFrag<PREC> load_a(const FacPtr& f, long long i, bool ok, long long safe);
template <>
__device__ __forceinline__ AFrag<P64> load_a<P64>(const FacPtr& f, long long i, bool ok, long long) {
  return {ok ? f.d[i] : 0.0};
}
template <>
__device__ __forceinline__ AFrag<PSPLIT> load_a<PSPLIT>(const FacPtr& f, long long i, bool ok, long long safe) {
  const float2 v = f.hl[ok ? i : safe];
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ AFrag<P32> load_a<P32>(const FacPtr& f, long long i, bool ok, long long safe) {
  const float2 v = f.hl[ok ? i : safe];
  return {v.x, v.y};
}

template <int PREC> struct BFrag;
template <> struct BFrag<P64> { double b; };
template <> struct BFrag<PSPLIT> { float b1, b2; };
template <> struct BFrag<P32> { float b; };

// sh = kSliceBits - e for the column's max |x| < 2^e (0 for an all-zero column).  The split
// form works in units of the column's grid 2^-sh: the leading slice is the integer
// x1 = rint(2^sh x) (|x1| <= 2^11, exact in FP32) and the remainder x2 = fp32(2^sh x - x1)
// (|x2| <= 1/2), so both stay normal FP32 numbers whatever the column's magnitude; the
// accumulators hold results in the same units and are scaled back when read (ldexp: exact,
// no scale can overflow).
template <int PREC>
__device__ __forceinline__ BFrag<PREC> make_b(double x, int sh);
template <>
__device__ __forceinline__ BFrag<P64> make_b<P64>(double x, int) { return {x}; }
template <>
__device__ __forceinline__ BFrag<PSPLIT> make_b<PSPLIT>(double x, int sh) {
  const double y = ldexp(x, sh);
  const double y1 = rint(y);
  return {static_cast<float>(y1), static_cast<float>(y - y1)};
}
template <>
__device__ __forceinline__ BFrag<P32> make_b<P32>(double x, int) { return {static_cast<float>(x)}; }

// Split form, for vector blocks that serve only as B operands: cut the rows x NT block (row
// stride LD) once per work-group, in place, into (x1, x2) float pairs on the column grids
// sh[c] (each double slot then holds one float2), instead of once per row tile in every wave.
template <int NT, int LD>
__device__ void cut_block(double* blk, int rows, const int* sh) {
  for (int e = threadIdx.x; e < rows * NT; e += 256) {
    const int r = e / NT, c = e % NT;
    double* q = blk + r * LD + c;
    const BFrag<PSPLIT> b = make_b<PSPLIT>(*q, sh[c]);
    *reinterpret_cast<float2*>(q) = make_float2(b.b1, b.b2);
  }
}

// B fragment of entry p[i] (0 where ok is false) from a block prepared for PREC: FP64 and
// FP32 values are converted here, the split form reads the pair left by cut_block.
template <int PREC>
__device__ __forceinline__ BFrag<PREC> b_from(const double* p, int i, bool ok, int sh) {
  if constexpr (PREC == PSPLIT) {
    const float2 v = ok ? *reinterpret_cast<const float2*>(p + i) : make_float2(0.0f, 0.0f);
    return {v.x, v.y};
  } else {
    return make_b<PREC>(sel_load<PREC>(p, i, ok, i), sh);
  }
}

// The NTL adjacent entries p[0 .. NTL) of a lane's columns (zeros where ok is false): one
// 16-byte load for two (p is 16-byte aligned), except in the branch-free FP32 form, where
// separate loads measured faster; p is readable when ok is false in that form.
template <int NTL, int PREC>
__device__ __forceinline__ void load_cols(const double* p, bool ok, double (&x)[NTL]) {
  if constexpr (NTL == 2 && !kBranchFree<PREC>) {
    const double2 v = ok ? *reinterpret_cast<const double2*>(p) : make_double2(0.0, 0.0);
    x[0] = v.x;
    x[1] = v.y;
  } else {
#pragma unroll
    for (int n = 0; n < NTL; ++n) x[n] = sel_load<PREC>(p, n, ok, n);
  }
}

// B fragments of a lane's NTL columns from a block prepared for PREC (see b_from).
template <int NTL, int PREC>
__device__ __forceinline__ void b_cols(const double* p, bool ok, const int (&sh)[NTL], BFrag<PREC> (&b)[NTL]) {
  if constexpr (PREC == PSPLIT && NTL == 2) {
    const float4 v = ok ? *reinterpret_cast<const float4*>(p) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    b[0] = {v.x, v.y};
    b[1] = {v.z, v.w};
  } else if constexpr (PREC == PSPLIT) {
#pragma unroll
    for (int n = 0; n < NTL; ++n) b[n] = b_from<PREC>(p, n, ok, sh[n]);
  } else {
    double x[NTL];
    load_cols<NTL, PREC>(p, ok, x);
#pragma unroll
    for (int n = 0; n < NTL; ++n) b[n] = make_b<PREC>(x[n], sh[n]);
  }
}

template <int PREC> struct Acc;
template <>
struct Acc<P64> {
  d4 v;
  __device__ void zero() { v = d4{0.0, 0.0, 0.0, 0.0}; }
  __device__ void set(int e, double x, int) { v[e] = x; }
  __device__ void step(const AFrag<P64>& a, const BFrag<P64>& b) { v = mfma64(a.a, b.b, v); }
  __device__ void flush_step() {}
  __device__ void flush() {}
  __device__ double get(int e, int) const { return v[e]; }
  __device__ void rescale(int) {}
};
template <>
struct Acc<PSPLIT> {
  d4 hi;
  f4 ex, cr;
  __device__ void zero() {
    hi = d4{0.0, 0.0, 0.0, 0.0};
    ex = f4{0.f, 0.f, 0.f, 0.f};
    cr = ex;
  }
  // sh: the shift of the lane's column (values held in units of 2^-sh, see make_b)
  __device__ void set(int e, double x, int sh) { hi[e] = ldexp(x, sh); }
  // one K-step (flushed after every K-step): the exact leading sum of four products, then
  // the corrections, smallest first
  __device__ void step(const AFrag<PSPLIT>& a, const BFrag<PSPLIT>& b) {
    ex = mfma32(a.a1, b.b1, ex);
    cr = mfma32(a.a2, b.b2, cr);
    cr = mfma32(a.a2, b.b1, cr);
    cr = mfma32(a.a1, b.b2, cr);
  }
  __device__ void flush_step() {
#pragma unroll
    for (int e = 0; e < 4; ++e) hi[e] += static_cast<double>(ex[e]) + static_cast<double>(cr[e]);
    ex = f4{0.f, 0.f, 0.f, 0.f};
    cr = ex;
  }
  __device__ void flush() {}
  __device__ double get(int e, int sh) const {
    return ldexp(hi[e] + static_cast<double>(ex[e]) + static_cast<double>(cr[e]), -sh);
  }
  // the column's grid moves from 2^-sh to 2^-(sh + d) (after a flush)
  __device__ void rescale(int d) {
#pragma unroll
    for (int e = 0; e < 4; ++e) hi[e] = ldexp(hi[e], d);
  }
};
template <>
struct Acc<P32> {
  d4 base;
  f4 v;
  __device__ void zero() {
    base = d4{0.0, 0.0, 0.0, 0.0};
    v = f4{0.f, 0.f, 0.f, 0.f};
  }
  __device__ void set(int e, double x, int) { base[e] = x; }
  __device__ void step(const AFrag<P32>& a, const BFrag<P32>& b) { v = mfma32(a.a1 + a.a2, b.b, v); }
  __device__ void flush_step() {}
  __device__ void flush() {}
  __device__ double get(int e, int) const { return base[e] + static_cast<double>(v[e]); }
  __device__ void rescale(int) {}
};

// Per-column slice shifts of a rows x NT block: sh[c] = kSliceBits - e, max |x| < 2^e.
// fetch(r, c) returns the FP64 entry.  All 256 threads take part; red must hold 256 doubles.
template <int NT, typename Fetch>
__device__ void column_scales(int rows, Fetch&& fetch, double* red, int* sc) {
  constexpr int GROUPS = 256 / NT;
  const int c = threadIdx.x % NT, g = threadIdx.x / NT;
  double mx = 0.0;
  for (int r = g; r < rows; r += GROUPS) mx = fmax(mx, fabs(fetch(r, c)));
  red[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x < NT) {
    double m = 0.0;
    for (int q = 0; q < GROUPS; ++q) m = fmax(m, red[q * NT + threadIdx.x]);
    int e = 0;
    if (m > 0.0) (void)frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
    sc[threadIdx.x] = m > 0.0 ? kSliceBits - e : 0;
  }
  __syncthreads();
}

// ------------------------------------------------------------------- level, synthesis
// One (task, column block): out_o = in[skel_o] + T_o in[red_o] for the task's outputs.  The
// input block is staged in `lds` (K x (NT + 2) doubles, one row of zeros, then the index
// lists).
template <int NT, int PREC, bool PIN = true>
__device__ void level_synth_body(const LevelTask& tk, int blk, const FacPtr& fp,
                                 const uint16_t* __restrict__ idx, const PairDesc* __restrict__ pairs,
                                 const double* __restrict__ in, double* __restrict__ out, int R,
                                 const CoefIO& io, double* lds) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  __shared__ double red_s[256];
  __shared__ int colsc[NT];
  const int K = tk.K;
  const long long c0 = static_cast<long long>(blk) * NT;
  double* xs = lds;                                                // K x LD, then row K = 0
  uint16_t* ix = reinterpret_cast<uint16_t*>(lds + (K + 1) * LD);  // [skel0 red0 skel1 red1]
  const int k0 = tk.k[0], k1 = tk.k[1] < 0 ? 0 : tk.k[1];
  // the zero row: the B operand of K-steps past the end of the contraction (no per-step mask)
  for (int c = threadIdx.x; c < LD; c += 256) xs[K * LD + c] = 0.0;
  if (io.on() && tk.mp >= 0) {
    const PairDesc pd = pairs[tk.mp];
    gather_leaf_block<NT, LD>(io, pd.m, pd.p, tk.in_row - pd.in_base, K, c0, xs);
  } else {
    stage_rows<NT, LD>(in + static_cast<long long>(tk.in_row) * R + c0, K, R, xs);
  }
  if (k0 > 0)
    for (int e = threadIdx.x; e < K; e += 256) ix[e] = idx[tk.idx[0] + e];
  if (k1 > 0)
    for (int e = threadIdx.x; e < K; e += 256) ix[(k0 > 0 ? K : 0) + e] = idx[tk.idx[1] + e];
  __syncthreads();
  if (PREC == PSPLIT)
    column_scales<NT>(K, [&](int r, int c) { return xs[r * LD + c]; }, red_s, colsc);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar registers
  const int lc = lane & 15, lr = lane >> 4;
  int bsc[NTL];
#pragma unroll
  for (int n = 0; n < NTL; ++n) bsc[n] = PREC == PSPLIT ? colsc[lc * NTL + n] : 0;
  const int nm0 = (k0 + 15) >> 4, nm1 = (k1 + 15) >> 4;
  const int np0 = (nm0 + 1) >> 1, np1 = (nm1 + 1) >> 1;  // pairs of row tiles per output
  for (int q = wave; q < np0 + np1; q += 4) {
    const int o = q < np0 ? 0 : 1;
    const int mt0 = 2 * (o ? q - np0 : q);
    const int k = o ? k1 : k0;
    const int nr = K - k;
    const uint16_t* skel = ix + (o && k0 > 0 ? K : 0);
    const uint16_t* red = skel + k;
    const long long toff = tk.fac[o];
    const bool two = mt0 + 1 < (o ? nm1 : nm0);
    Acc<PREC> acc[2][NTL];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        acc[u][n].zero();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (mt0 + u) * 16 + drow<PREC>(v, lr);
          acc[u][n].set(v, row < k ? xs[skel[row] * LD + lc * NTL + n] : 0.0, bsc[n]);
        }
      }
    }
    const int i0 = mt0 * 16 + lc, i1 = i0 + 16;
    // factor fragments are fetched PF K-steps ahead (double-buffered in registers), and with
    // them the LDS row offsets of the gathered vector rows, so that a K-step waits on one LDS
    // read instead of two dependent ones
    // K-steps fetched ahead: the persistent kernel and the split form take half (fewer
    // registers: the split 16-column kernel fits five waves per SIMD, which measured faster)
    constexpr int PF = (PIN && PREC != PSPLIT) ? kPrefetch : kPrefetch / 2;
    const int nsteps = (nr + 3) >> 2;
    // The K loop is compiled twice, for a pair of row tiles and for a lone tile, so that the
    // pair's matrix instructions run without a branch between them.
    auto kloop = [&](auto tiles) {
    constexpr int TC = decltype(tiles)::value;
    const bool TWO = TC == 2 ? two : TC == 1;
    AFrag<PREC> a0c[PF], a1c[PF], a0n[PF], a1n[PF];
    int roc[PF], ron[PF];
    auto fetch = [&](int s0, AFrag<PREC>* d0, AFrag<PREC>* d1, int* ro) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int kk = (s0 + u) * 4 + lr;
        const bool kin = kk < nr;
        const long long base = toff + static_cast<long long>(kk) * k;
        d0[u] = load_a<PREC>(fp, base + i0, kin && i0 < k, toff);
        if (TWO || kBranchFree<PREC>) d1[u] = load_a<PREC>(fp, base + i1, kin && TWO && i1 < k, toff);
        ro[u] = (kin ? red[kk] : K) * LD;
      }
    };
    // Each block's fragments are taken over at the top of the loop (the only wait on their
    // loads, issued one block earlier), then the next block's loads are issued; the
    // scheduling barrier (PIN) keeps the compiler from sinking them towards their use.  The
    // persistent batch kernel leaves the placement to the compiler: there the barrier raised
    // its register use and slowed it down.  The unmasked loads read the block's first entry,
    // which exists only when there is a step.
    if (nsteps > 0) fetch(0, a0n, a1n, ron);
    for (int s0 = 0; s0 < nsteps; s0 += PF) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        a0c[u] = a0n[u];
        a1c[u] = a1n[u];
        roc[u] = ron[u];
      }
      if (s0 + PF < nsteps) fetch(s0 + PF, a0n, a1n, ron);
      if (PIN) __builtin_amdgcn_sched_barrier(0);  // the next block's loads stay where they are issued
      // the vector rows are read one K-step ahead (steps past the end read the zero row)
      double xb[2][NTL];
      load_cols<NTL, PREC>(xs + roc[0] + lc * NTL, true, xb[0]);
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (u + 1 < PF) load_cols<NTL, PREC>(xs + roc[u + 1] + lc * NTL, true, xb[(u + 1) & 1]);
        const double* xv = xb[u & 1];
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          const BFrag<PREC> b = make_b<PREC>(xv[n], bsc[n]);
          acc[0][n].step(a0c[u], b);
          // a lone tile's partner rows are never stored; the branch-free form computes them
          if (kBranchFree<PREC> || TWO) acc[1][n].step(a1c[u], b);
        }
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          acc[0][n].flush_step();
          if (TWO) acc[1][n].flush_step();
        }
      }
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        acc[0][n].flush();
        acc[1][n].flush();
      }
    }
    };
    if (two)
      kloop(TileCount<1>{});
    else
      kloop(TileCount<0>{});
    double* ob = out + static_cast<long long>(tk.out_row[o]) * R + c0 + lc * NTL;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (mt0 + u) * 16 + drow<PREC>(v, lr);
        if (row < k) {
#pragma unroll
          for (int n = 0; n < NTL; ++n) ob[static_cast<long long>(row) * R + n] = acc[u][n].get(v, bsc[n]);
        }
      }
    }
  }
}

template <int NT, int PREC>
__global__ void __launch_bounds__(256, kMinBlocks)
k_level_synth_mfma(const LevelTask* __restrict__ tasks, long long ntasks, int nblk, FacPtr fp,
                   const uint16_t* __restrict__ idx, const PairDesc* __restrict__ pairs,
                   const double* __restrict__ in, double* __restrict__ out, int R, CoefIO io) {
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  level_synth_body<NT, PREC>(tasks[ti], blk, fp, idx, pairs, in, out, R, io, lds);
}

// The split 16-column form held to six waves per SIMD (80 VGPRs).
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(6, 8)))
k_level_synth_split6(const LevelTask* __restrict__ tasks, long long ntasks, int nblk, FacPtr fp,
                     const uint16_t* __restrict__ idx, const PairDesc* __restrict__ pairs,
                     const double* __restrict__ in, double* __restrict__ out, int R, CoefIO io) {
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  level_synth_body<16, PSPLIT>(tasks[ti], blk, fp, idx, pairs, in, out, R, io, lds);
}

// ------------------------------------------------------------------ level, transposed
// Output block o contributes T_o^T w_o at rows red_o and w_o at rows skel_o; every input row
// gets exactly one term from each block.  Both blocks run at once (their row-tile pairs are
// dealt to the waves together, as in the synthesis kernel) and every term is added into the
// zeroed LDS block with an LDS atomic add: a row receives at most two terms, and 0 + a + b
// gives the same bits in either order, so the result does not depend on timing.
// LDS: the accumulated input block (K x NT), for the split form the vectors w_0 and w_1
// (k_0 + k_1 rows, cut on the fly from their own column scales), then the index lists.  FP64
// and FP32 read w_o as B fragments straight from global memory (prefetched with the factor
// fragments): their loops are not VALU-bound and the smaller LDS block keeps 32-column tiles.
// The split form does the same (WLDS = false) for size classes whose LDS block would
// otherwise leave room for only one work-group per compute unit.
template <int NT, int PREC, bool WLDS = PREC == PSPLIT, bool PIN = true>
__device__ void level_trans_body(const LevelTask& tk, int blk, const FacPtr& fp,
                                 const uint16_t* __restrict__ idx, const PairDesc* __restrict__ pairs,
                                 const double* __restrict__ win, double* __restrict__ xout, int R,
                                 const CoefIO& io, double* lds) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  __shared__ double red_s[256];
  __shared__ int colsc[2][NT];
  const int K = tk.K;
  const long long c0 = static_cast<long long>(blk) * NT;
  const int nouts = tk.k[1] < 0 ? 1 : 2;
  const int k0 = tk.k[0], k1 = tk.k[1] < 0 ? 0 : tk.k[1];
  double* acc_l = lds;
  double* wl0 = acc_l + K * LD;
  double* wl1 = wl0 + (WLDS ? k0 * LD : 0);
  uint16_t* ix = reinterpret_cast<uint16_t*>(wl1 + (WLDS ? k1 * LD : 0));  // [skel0 red0 skel1 red1]
  for (int o = 0; o < nouts; ++o)
    for (int e = threadIdx.x; e < K; e += 256) ix[o * K + e] = idx[tk.idx[o] + e];
  for (int e = threadIdx.x; e < K * LD; e += 256) acc_l[e] = 0.0;
  const double* wg0 = win + static_cast<long long>(tk.out_row[0]) * R + c0;
  const double* wg1 = win + static_cast<long long>(nouts > 1 ? tk.out_row[1] : tk.out_row[0]) * R + c0;
  if (WLDS) {
    stage_rows<NT, LD>(wg0, k0, R, wl0);
    if (nouts > 1) stage_rows<NT, LD>(wg1, k1, R, wl1);
  }
  __syncthreads();
  if (PREC == PSPLIT) {
    if (WLDS) {
      column_scales<NT>(k0, [&](int r, int c) { return wl0[r * LD + c]; }, red_s, colsc[0]);
      if (nouts > 1) column_scales<NT>(k1, [&](int r, int c) { return wl1[r * LD + c]; }, red_s, colsc[1]);
    } else {
      column_scales<NT>(k0, [&](int r, int c) { return wg0[static_cast<long long>(r) * R + c]; }, red_s,
                        colsc[0]);
      if (nouts > 1)
        column_scales<NT>(k1, [&](int r, int c) { return wg1[static_cast<long long>(r) * R + c]; }, red_s,
                          colsc[1]);
    }
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar registers
  const int lc = lane & 15, lr = lane >> 4;
  const int nm0 = (K - k0 + 15) >> 4, nm1 = nouts > 1 ? (K - k1 + 15) >> 4 : 0;
  const int np0 = (nm0 + 1) >> 1, np1 = (nm1 + 1) >> 1;  // pairs of row tiles per output
  for (int q = wave; q < np0 + np1; q += 4) {
    const int o = q < np0 ? 0 : 1;
    const int mt0 = 2 * (o ? q - np0 : q);
    const int k = o ? k1 : k0;
    const int nr = K - k;
    const bool two = mt0 + 1 < (o ? nm1 : nm0);
    const uint16_t* red = ix + o * K + k;
    const long long toff = tk.fac[o];  // T^T: nr x k column-major
    const double* wg = o ? wg1 : wg0;
    const double* wl = o ? wl1 : wl0;
    int bsc[NTL];
#pragma unroll
    for (int n = 0; n < NTL; ++n) bsc[n] = PREC == PSPLIT ? colsc[o][lc * NTL + n] : 0;
    Acc<PREC> acc[2][NTL];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int n = 0; n < NTL; ++n) acc[u][n].zero();
    const int j0 = mt0 * 16 + lc, j1 = j0 + 16;
    // K-steps fetched ahead: half in the persistent kernel and in the split form that reads its
    // vectors from global memory (fewer registers, four waves per SIMD)
    constexpr int PF = (PIN && (WLDS || PREC != PSPLIT)) ? kPrefetch : kPrefetch / 2;
    const int nsteps = (k + 3) >> 2;
    // compiled for a pair of row tiles and for a lone tile (no branch between the pair's
    // matrix instructions), as in the synthesis kernel; FP64 keeps one loop with the test at
    // run time, which measured faster for it (1.4 ms per step at l = 1024, 64 fields)
    auto kloop = [&](auto tiles) {
    constexpr int TC = decltype(tiles)::value;
    const bool TWO = TC == 2 ? two : TC == 1;
    AFrag<PREC> a0c[PF], a1c[PF], a0n[PF], a1n[PF];
    constexpr int PB = WLDS ? 1 : PF;  // B fragments prefetched with A when read from global
    double bc[PB][NTL], bn[PB][NTL];
    auto fetch = [&](int s0, AFrag<PREC>* d0, AFrag<PREC>* d1, double (*b)[NTL]) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int i = (s0 + u) * 4 + lr;
        const bool iin = i < k;
        const long long base = toff + static_cast<long long>(i) * nr;
        d0[u] = load_a<PREC>(fp, base + j0, iin && j0 < nr, toff);
        if (TWO || kBranchFree<PREC>) d1[u] = load_a<PREC>(fp, base + j1, iin && TWO && j1 < nr, toff);
        if (!WLDS)  // (branch-free: row 0 stands in for rows past the block)
          load_cols<NTL, PREC>(wg + static_cast<long long>(kBranchFree<PREC> && !iin ? 0 : i) * R + lc * NTL, iin,
                               b[u % PB]);
      }
    };
    if (nsteps > 0) fetch(0, a0n, a1n, bn);
    for (int s0 = 0; s0 < nsteps; s0 += PF) {  // (the block hand-over of the synthesis loop)
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        a0c[u] = a0n[u];
        a1c[u] = a1n[u];
      }
      if (!WLDS) {
#pragma unroll
        for (int u = 0; u < PB; ++u)
#pragma unroll
          for (int n = 0; n < NTL; ++n) bc[u][n] = bn[u][n];
      }
      if (s0 + PF < nsteps) fetch(s0 + PF, a0n, a1n, bn);
      if (PIN) __builtin_amdgcn_sched_barrier(0);  // the next block's loads stay where they are issued
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int i = (s0 + u) * 4 + lr;
        const bool iin = i < k;
        double xv[NTL];
        if (WLDS) load_cols<NTL, PREC>(wl + (iin ? i : 0) * LD + lc * NTL, iin, xv);
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          const BFrag<PREC> b = make_b<PREC>(WLDS ? xv[n] : bc[u % PB][n], bsc[n]);
          acc[0][n].step(a0c[u], b);
          if (kBranchFree<PREC> || TWO) acc[1][n].step(a1c[u], b);
        }
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          acc[0][n].flush_step();
          if (TWO) acc[1][n].flush_step();
        }
      }
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        acc[0][n].flush();
        acc[1][n].flush();
      }
    }
    };
    if constexpr (PREC == P64) {
      kloop(TileCount<2>{});
    } else {
      if (two)
        kloop(TileCount<1>{});
      else
        kloop(TileCount<0>{});
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = (mt0 + u) * 16 + drow<PREC>(v, lr);
        if (j < nr) {
          double* dst = acc_l + static_cast<int>(red[j]) * LD + lc * NTL;
#pragma unroll
          for (int n = 0; n < NTL; ++n) atomicAdd(dst + n, acc[u][n].get(v, bsc[n]));
        }
      }
    }
  }
  // identity part: w_o at the skeleton rows of each block
  for (int o = 0; o < nouts; ++o) {
    const int k = o ? k1 : k0;
    const uint16_t* skel = ix + o * K;
    if (WLDS) {
      const double* wl = o ? wl1 : wl0;
      for (int e = threadIdx.x; e < k * NT; e += 256) {
        const int i = e / NT, c = e % NT;
        atomicAdd(acc_l + static_cast<int>(skel[i]) * LD + c, wl[i * LD + c]);
      }
    } else {
      const double* wg = o ? wg1 : wg0;
      staged<double>(
          k * NT, [&](int e) { return wg[static_cast<long long>(e / NT) * R + e % NT]; },
          [&](int e, double val) { atomicAdd(acc_l + static_cast<int>(skel[e / NT]) * LD + e % NT, val); });
    }
  }
  __syncthreads();
  if (io.on() && tk.mp >= 0) {
    const PairDesc pd = pairs[tk.mp];
    for_leaf_block<NT>(io, pd.m, pd.p, tk.in_row - pd.in_base, K, c0,
                       [&](int j, int c, double* a, bool imag0) {
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

template <int NT, int PREC, bool WLDS = PREC == PSPLIT>
__global__ void __launch_bounds__(256, kMinBlocks)
k_level_trans_mfma(const LevelTask* __restrict__ tasks, long long ntasks, int nblk, FacPtr fp,
                   const uint16_t* __restrict__ idx, const PairDesc* __restrict__ pairs,
                   const double* __restrict__ win, double* __restrict__ xout, int R, CoefIO io) {
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  level_trans_body<NT, PREC, WLDS>(tasks[ti], blk, fp, idx, pairs, win, xout, R, io, lds);
}

// The split form with vectors read from global memory, held to 96 VGPRs (one fewer than it
// takes unconstrained): five waves per SIMD where the LDS block allows five work-groups.
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(5, 8)))
k_level_trans_split_g(const LevelTask* __restrict__ tasks, long long ntasks, int nblk, FacPtr fp,
                      const uint16_t* __restrict__ idx, const PairDesc* __restrict__ pairs,
                      const double* __restrict__ win, double* __restrict__ xout, int R, CoefIO io) {
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  level_trans_body<16, PSPLIT, false>(tasks[ti], blk, fp, idx, pairs, win, xout, R, io, lds);
}

// ------------------------------------------------------------------- final, synthesis
// E = S_0 v_0, O = S_1 v_1 on one 16-row tile; g(+-x) = (E +- O) / D.
template <int NT, int PREC, bool PIN = true>
__device__ void final_synth_body(const FinalTask& ft, int blk, const FacPtr& fp,
                                 const double* __restrict__ v0buf, const double* __restrict__ v1buf,
                                 const double* __restrict__ invD, double* __restrict__ Y, int l, int R,
                                 double* lds) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  __shared__ double red_s[256];
  __shared__ int colsc[2][NT];
  const long long c0 = static_cast<long long>(blk) * NT;
  const double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1], h = ft.h;
  double* w0 = lds;
  double* w1 = lds + k0 * LD;
  stage_rows<NT, LD>(V + static_cast<long long>(ft.in_row[0]) * R + c0, k0, R, w0);
  stage_rows<NT, LD>(V + static_cast<long long>(ft.in_row[1]) * R + c0, k1, R, w1);
  __syncthreads();
  if (PREC == PSPLIT) {
    column_scales<NT>(k0, [&](int r, int c) { return w0[r * LD + c]; }, red_s, colsc[0]);
    column_scales<NT>(k1, [&](int r, int c) { return w1[r * LD + c]; }, red_s, colsc[1]);
    cut_block<NT, LD>(w0, k0, colsc[0]);
    cut_block<NT, LD>(w1, k1, colsc[1]);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar registers
  const int lc = lane & 15, lr = lane >> 4;
  int bsc[2][NTL];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int n = 0; n < NTL; ++n) bsc[p][n] = PREC == PSPLIT ? colsc[p][lc * NTL + n] : 0;
  const int nm = (h + 15) >> 4;
  for (int mt = wave; mt < nm; mt += 4) {
    Acc<PREC> E[NTL], O[NTL];
#pragma unroll
    for (int n = 0; n < NTL; ++n) {
      E[n].zero();
      O[n].zero();
    }
    const int i = mt * 16 + lc;
    const bool iin = i < h;
    // both parities in one prefetched loop, interleaved: step st feeds E (rows of S_0) and O
    // (rows of S_1) at once, two independent accumulator chains per wave
    constexpr int PF = PIN ? kPrefetch / 2 : kPrefetch / 4;
    const int n0 = (k0 + 3) >> 2, n1 = (k1 + 3) >> 2, nsteps = n0 > n1 ? n0 : n1;
    const long long safe = k0 > 0 ? ft.fac[0] : ft.fac[1];  // a non-empty block when nsteps > 0
    AFrag<PREC> ec[PF], en[PF], oc[PF], on[PF];
    auto fetch = [&](int s0) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int a = (s0 + u) * 4 + lr;
        en[u] = load_a<PREC>(fp, ft.fac[0] + static_cast<long long>(a) * h + i, a < k0 && iin, safe);
        on[u] = load_a<PREC>(fp, ft.fac[1] + static_cast<long long>(a) * h + i, a < k1 && iin, safe);
      }
    };
    if (nsteps > 0) fetch(0);
    for (int s0 = 0; s0 < nsteps; s0 += PF) {  // (the block hand-over of the level loops)
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        ec[u] = en[u];
        oc[u] = on[u];
      }
      if (s0 + PF < nsteps) fetch(s0 + PF);
      if (PIN) __builtin_amdgcn_sched_barrier(0);  // the next block's loads stay where they are issued
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int a = (s0 + u) * 4 + lr;
        const bool a0 = a < k0, a1 = a < k1;
        BFrag<PREC> be[NTL], bo[NTL];
        b_cols<NTL, PREC>(w0 + (a0 ? a : 0) * LD + lc * NTL, a0, bsc[0], be);
        b_cols<NTL, PREC>(w1 + (a1 ? a : 0) * LD + lc * NTL, a1, bsc[1], bo);
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          E[n].step(ec[u], be[n]);
          O[n].step(oc[u], bo[n]);
        }
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          E[n].flush_step();
          O[n].flush_step();
        }
      }
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        E[n].flush();
        O[n].flush();
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ii = mt * 16 + drow<PREC>(v, lr);
      if (ii < h) {
        const int row = ft.row0 + ii;
        const double s = invD[row];
        double* yp = Y + y_row(l, ft.m, l + row) * R + c0 + lc * NTL;
        double* ym = Y + y_row(l, ft.m, l - 1 - row) * R + c0 + lc * NTL;
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          const double e = E[n].get(v, bsc[0][n]), od = O[n].get(v, bsc[1][n]);
          yp[n] = (e + od) * s;
          ym[n] = (e - od) * s;
        }
      }
    }
  }
}

template <int NT, int PREC>
__global__ void __launch_bounds__(256, kMinBlocks)
k_final_synth_mfma(const FinalTask* __restrict__ tasks, long long ntasks, int nblk, FacPtr fp,
                   const double* __restrict__ v0buf, const double* __restrict__ v1buf,
                   const double* __restrict__ invD, double* __restrict__ Y, int l, int R) {
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  final_synth_body<NT, PREC>(tasks[ti], blk, fp, v0buf, v1buf, invD, Y, l, R, lds);
}

// ------------------------------------------------------------------ final, transposed
// v_p = S_p^T (half * scale * (G(+x) +- G(-x))): the folded rows are built in LDS chunk by
// chunk; each wave keeps the accumulators of its row tiles across the chunks.
// LDS: the two folded chunks, 2 x ICH x (NT + 2) doubles.
template <int NT, int ICH>
constexpr size_t final_trans_lds() { return 2 * ICH * ldp<NT>() * sizeof(double); }

template <int NT, int ICH, int PREC, bool PIN = true, int MAXT = 6>
__device__ void final_trans_body(const FinalTask& ft, int blk, const FacPtr& fp,
                                 const double* __restrict__ Yin, const double* __restrict__ scale,
                                 double half, double* __restrict__ v0buf, double* __restrict__ v1buf,
                                 int l, int R, double* lds) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  // MAXT: output tiles per wave and pass (a pass covers 4 MAXT tiles, 64 MAXT rows); even
  static_assert(MAXT % 2 == 0, "output tiles go through the rows in pairs");
  double* eo[2] = {lds, lds + ICH * LD};
  __shared__ double red_s[256];
  __shared__ int colsc[2][NT];
  const long long c0 = static_cast<long long>(blk) * NT;
  double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1], h = ft.h;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar registers
  const int lc = lane & 15, lr = lane >> 4;
  const int nm0 = (k0 + 15) >> 4, nm1 = (k1 + 15) >> 4;
  // Output tiles [0, nm0 + nm1) are covered in passes of 4 MAXT tiles (the accumulators one
  // wave keeps in registers); ranks k0 + k1 above 64 MAXT take more than one pass over the
  // rows, each staging the folded rows again.
  for (int t0 = 0; t0 < nm0 + nm1; t0 += 4 * MAXT) {
  Acc<PREC> acc[MAXT][NTL];
#pragma unroll
  for (int u = 0; u < MAXT; ++u)
#pragma unroll
    for (int n = 0; n < NTL; ++n) acc[u][n].zero();
  // split form: each row chunk has its own column grids; the sums so far move to the new grid
  int shp[2][NTL] = {};
  for (int i0 = 0; i0 < h; i0 += ICH) {
    const int ih = min(ICH, h - i0);
    __syncthreads();
    // two items in flight: the accumulator tiles of the pass stay live in registers meanwhile
    staged<double2, 2>(
        ih * NT,
        [&](int e) {
          const int row = ft.row0 + i0 + e / NT, c = e % NT;
          return make_double2(Yin[y_row(l, ft.m, l + row) * R + c0 + c], Yin[y_row(l, ft.m, l - 1 - row) * R + c0 + c]);
        },
        [&](int e, double2 g) {
          const int i = e / NT, c = e % NT;
          const double sc = half * scale[ft.row0 + i0 + i];
          eo[0][i * LD + c] = (g.x + g.y) * sc;
          eo[1][i * LD + c] = (g.x - g.y) * sc;
        });
    __syncthreads();
    if (PREC == PSPLIT) {
      column_scales<NT>(ih, [&](int r, int c) { return eo[0][r * LD + c]; }, red_s, colsc[0]);
      column_scales<NT>(ih, [&](int r, int c) { return eo[1][r * LD + c]; }, red_s, colsc[1]);
      cut_block<NT, LD>(eo[0], ih, colsc[0]);
      cut_block<NT, LD>(eo[1], ih, colsc[1]);
      __syncthreads();
#pragma unroll
      for (int u = 0; u < MAXT; ++u) {
        const int pu = t0 + wave + 4 * u < nm0 ? 0 : 1;
#pragma unroll
        for (int n = 0; n < NTL; ++n) acc[u][n].rescale(colsc[pu][lc * NTL + n] - shp[pu][n]);
      }
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int n = 0; n < NTL; ++n) shp[pp][n] = colsc[pp][lc * NTL + n];
    }
    // Two output tiles per pass through the rows, so that one tile's matrix instructions
    // overlap the other's accumulator hand-over (the split form flushes after every K-step);
    // a wave's last tile, when it has no partner, runs a loop of its own.
#pragma unroll
    for (int u = 0; u < MAXT; u += 2) {
      const int q0 = t0 + wave + 4 * u;  // tile index over [output 0 tiles | output 1 tiles]
      if (q0 >= nm0 + nm1) break;
      const int q1 = q0 + 4 < nm0 + nm1 ? q0 + 4 : q0;
      const int p0 = q0 < nm0 ? 0 : 1, p1 = q1 < nm0 ? 0 : 1;
      const int kk0 = p0 ? k1 : k0, kk1 = p1 ? k1 : k0;
      const int a0 = (p0 ? q0 - nm0 : q0) * 16 + lc, a1 = (p1 ? q1 - nm0 : q1) * 16 + lc;
      const long long so0 = ft.fac[p0], so1 = ft.fac[p1];  // S^T: k x h column-major
      const double* src0 = eo[p0];
      const double* src1 = eo[p1];
      int bs0[NTL], bs1[NTL];
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
        bs0[n] = PREC == PSPLIT ? colsc[p0][lc * NTL + n] : 0;
        bs1[n] = PREC == PSPLIT ? colsc[p1][lc * NTL + n] : 0;
      }
      constexpr int PF = PIN ? kPrefetch / 2 : kPrefetch / 4;
      const int nsteps = (ih + 3) >> 2;
      auto kloop = [&](auto tiles) __attribute__((always_inline)) {
        constexpr bool TWO = decltype(tiles)::value == 1;
        AFrag<PREC> ac0[PF], an0[PF], ac1[PF], an1[PF];
        auto fetch = [&](int s0) {
#pragma unroll
          for (int w = 0; w < PF; ++w) {
            const int i = (s0 + w) * 4 + lr;
            an0[w] = load_a<PREC>(fp, so0 + static_cast<long long>(i0 + i) * kk0 + a0, i < ih && a0 < kk0, so0);
            if (TWO)
              an1[w] = load_a<PREC>(fp, so1 + static_cast<long long>(i0 + i) * kk1 + a1, i < ih && a1 < kk1, so1);
          }
        };
        if (nsteps > 0) fetch(0);
        for (int s0 = 0; s0 < nsteps; s0 += PF) {  // (the block hand-over of the level loops)
#pragma unroll
          for (int w = 0; w < PF; ++w) {
            ac0[w] = an0[w];
            if (TWO) ac1[w] = an1[w];
          }
          if (s0 + PF < nsteps) fetch(s0 + PF);
          if (PIN) __builtin_amdgcn_sched_barrier(0);  // the next block's loads stay where they are issued
          // the folded rows are read from LDS one K-step ahead
          BFrag<PREC> bb[2][2][NTL];
          auto read_b = [&](int w, BFrag<PREC> (&b0)[NTL], BFrag<PREC> (&b1)[NTL]) {
            const int i = (s0 + w) * 4 + lr;
            const bool iin = i < ih;
            const double* e0 = src0 + (iin ? i : 0) * LD + lc * NTL;
            const double* e1 = src1 + (iin ? i : 0) * LD + lc * NTL;
#pragma unroll
            for (int n = 0; n < NTL; ++n) {
              b0[n] = b_from<PREC>(e0, n, iin, bs0[n]);
              if (TWO) b1[n] = b_from<PREC>(e1, n, iin, bs1[n]);
            }
          };
          read_b(0, bb[0][0], bb[0][1]);
#pragma unroll
          for (int w = 0; w < PF; ++w) {
            if (w + 1 < PF) read_b(w + 1, bb[(w + 1) & 1][0], bb[(w + 1) & 1][1]);
#pragma unroll
            for (int n = 0; n < NTL; ++n) {
              acc[u][n].step(ac0[w], bb[w & 1][0][n]);
              if (TWO) acc[u + 1][n].step(ac1[w], bb[w & 1][1][n]);
            }
#pragma unroll
            for (int n = 0; n < NTL; ++n) {
              acc[u][n].flush_step();
              if (TWO) acc[u + 1][n].flush_step();
            }
          }
#pragma unroll
          for (int n = 0; n < NTL; ++n) {
            acc[u][n].flush();
            if (TWO) acc[u + 1][n].flush();
          }
        }
      };
      if (q1 != q0)
        kloop(TileCount<1>{});
      else
        kloop(TileCount<0>{});
    }
  }
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    const int q = t0 + wave + 4 * u;
    if (q >= nm0 + nm1) break;
    const int p = q < nm0 ? 0 : 1;
    const int k = p ? k1 : k0;
    const int mt = p ? q - nm0 : q;
    double* vout = V + static_cast<long long>(ft.in_row[p]) * R + c0 + lc * NTL;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = mt * 16 + drow<PREC>(v, lr);
      if (a < k) {
#pragma unroll
        for (int n = 0; n < NTL; ++n)
          vout[static_cast<long long>(a) * R + n] = acc[u][n].get(v, PREC == PSPLIT ? colsc[p][lc * NTL + n] : 0);
      }
    }
  }
  }  // passes over the output tiles
}

template <int NT, int ICH, int PREC>
__global__ void __launch_bounds__(256, kMinBlocks)
k_final_trans_mfma(const FinalTask* __restrict__ tasks, long long ntasks, int nblk, FacPtr fp,
                   const double* __restrict__ Yin, const double* __restrict__ scale, double half,
                   double* __restrict__ v0buf, double* __restrict__ v1buf, int l, int R) {
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  // output tiles per wave and pass: fewer accumulators, more resident waves (split: two tiles,
  // 128 VGPRs, four waves per SIMD; FP64: four tiles, 124 VGPRs); larger ranks take more passes
  final_trans_body<NT, ICH, PREC, true, (PREC == PSPLIT ? 2 : 4)>(tasks[ti], blk, fp, Yin, scale, half, v0buf,
                                                                   v1buf, l, R, lds);
}

// ------------------------------------------------------------------ factor preparation
__global__ void k_transpose_blocks(const double* __restrict__ fac, double* __restrict__ fac_t,
                                   const FactorBlock* __restrict__ blocks) {
  const FactorBlock b = blocks[blockIdx.x];
  const long long n = static_cast<long long>(b.rows) * b.cols;
  for (long long e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = static_cast<int>(e % b.rows), c = static_cast<int>(e / b.rows);
    fac_t[b.off + static_cast<long long>(r) * b.cols + c] = fac[b.off + e];
  }
}

// Row-aligned split of every stored matrix (column-major, `rows` x `cols`; transposed: the
// stored block is cols x rows): hi = leading slice on the row's grid, lo = fp32 remainder.
__global__ void k_split_rows(const double* __restrict__ src, float2* __restrict__ hl,
                             const FactorBlock* __restrict__ blocks, int transposed) {
  const FactorBlock b = blocks[blockIdx.x];
  const int nrows = transposed ? b.cols : b.rows;
  const int ncols = transposed ? b.rows : b.cols;
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
    double mx = 0.0;
    for (int c = 0; c < ncols; ++c) mx = fmax(mx, fabs(src[b.off + static_cast<long long>(c) * nrows + r]));
    int e = 0;
    if (mx > 0.0) (void)frexp(mx, &e);
    const int sh = mx > 0.0 ? kSliceBits - e : 0;
    for (int c = 0; c < ncols; ++c) {
      const long long i = b.off + static_cast<long long>(c) * nrows + r;
      const double x = src[i];
      const double x1 = ldexp(rint(ldexp(x, sh)), -sh);
      hl[i] = make_float2(static_cast<float>(x1), static_cast<float>(x - x1));
    }
  }
}

// LDS budget (bytes) under which a level or final launch takes 32-column tiles instead of 16:
// a larger tile halves the factor reads per task, but only while two work-groups still fit
// in a compute unit's 160 KiB of LDS (a 16-column tile at two work-groups per CU measured
// faster than a 32-column tile at one).  SHT_TILE32_LDS_KB overrides it (tuning).
long long tile32_lds_budget() {
  static const long long v = [] {
    const char* e = std::getenv("SHT_TILE32_LDS_KB");
    const long long kb = e ? std::atoll(e) : 76;
    return (kb > 0 ? kb : 76) * 1024;
  }();
  return v;
}

// Largest LDS block (bytes) for which the transposed split levels stage their output vectors
// in LDS; 0 by default: the form that reads them from global memory (k_level_trans_split_g:
// 96 VGPRs and a small LDS block, five waves per SIMD) measured faster for every size class.
// SHT_SPLIT_WLDS_KB (tuning) sets a positive cap in KiB.
long long split_wlds_cap() {
  static const long long v = [] {
    const char* e = std::getenv("SHT_SPLIT_WLDS_KB");
    const long long kb = e ? std::atoll(e) : 0;
    return (kb > 0 ? kb : 0) * 1024;
  }();
  return v;
}

FacPtr fac_ptr(const sht_plan_s* P, bool transposed) {
  return transposed ? FacPtr{P->d.fac_t, P->d.fac_t_hl} : FacPtr{P->d.fac, P->d.fac_hl};
}

template <int PREC>
hipError_t level_class(const sht_plan_s* P, int step, const LaunchClass& lc, bool transpose,
                       const double* in, double* out, int R, const CoefIO& io, hipStream_t s) {
  const long long cnt = lc.cnt;
  if (cnt == 0) return hipSuccess;
  const LevelTask* tasks = P->d.tasks + P->step_off[step] + lc.off;
  const int K = lc.maxK;
  // LDS holds the task's K x NT input block: 32 columns while that stays within the tile
  // budget.  The split form always takes 16 columns: its 16-column kernels fit more waves
  // per SIMD in registers, which measured faster than the halved factor reads of 32 (FP64
  // measured the other way).  The transposed split form stages both output blocks only
  // where split_wlds_cap() allows (by default nowhere: the vectors are read from global
  // memory).
  bool wlds = false;
  long long rows = K;
  if (transpose && PREC == PSPLIT) {
    const long long rw = K + 2LL * lc.maxk;
    wlds = rw * 18 * 8 + 4LL * K + 16 <= split_wlds_cap();
    if (wlds) rows = rw;
  }
  const int NT = (PREC != PSPLIT && R % 32 == 0 && rows * 34 * 8 <= tile32_lds_budget()) ? 32 : 16;
  if ((rows + 1) * 18 * 8 + 4LL * K + 16 > 150 * 1024) return hipErrorInvalidConfiguration;
  const int nblk = R / NT;
  const dim3 grid(xcd_grid(cnt, nblk));
  const size_t lds = static_cast<size_t>(rows + 1) * (NT + 2) * 8 + 4 * static_cast<size_t>(K) + 16;
  const FacPtr fp = fac_ptr(P, transpose);
  hipError_t e;
#define LEVEL_LAUNCH(KER)                                                                              \
  do {                                                                                                 \
    if ((e = allow_lds(reinterpret_cast<const void*>(&KER), lds)) != hipSuccess) return e;             \
    hipLaunchKernelGGL(KER, grid, dim3(256), lds, s, tasks, cnt, nblk, fp, P->d.idx, P->d.pairs, in, out, \
                       R, io);                                                                          \
  } while (0)
  if (!transpose) {
    if (NT == 32)
      LEVEL_LAUNCH((k_level_synth_mfma<32, PREC>));
    else
      if constexpr (PREC == PSPLIT)
        LEVEL_LAUNCH(k_level_synth_split6);
      else
        LEVEL_LAUNCH((k_level_synth_mfma<16, PREC>));
  } else if (PREC == PSPLIT && !wlds) {
    if constexpr (PREC == PSPLIT)
      LEVEL_LAUNCH(k_level_trans_split_g);
    else
      LEVEL_LAUNCH((k_level_trans_mfma<16, PREC, false>));
  } else {
    if (NT == 32)
      LEVEL_LAUNCH((k_level_trans_mfma<32, PREC>));
    else
      LEVEL_LAUNCH((k_level_trans_mfma<16, PREC>));
  }
#undef LEVEL_LAUNCH
  return hipGetLastError();
}

template <int PREC>
hipError_t final_launch(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                        double* v0w, double* v1w, double* y, const double* yin, int R, bool adjoint,
                        hipStream_t s, int only) {
  hipError_t e;
  const FacPtr fp = fac_ptr(P, transpose);
  if (!transpose) {
    for (size_t c = 0; c < P->final_classes.size(); ++c) {
      if (only >= 0 && static_cast<int>(c) != only) continue;
      const LaunchClass& lc = P->final_classes[c];
      const long long cnt = lc.cnt;
      const FinalTask* tasks = P->d.finals + lc.off;
      const long long rows = 2LL * lc.maxk;
      const int NT =
          (PREC != PSPLIT && R % 32 == 0 && rows * 34 * 8 <= std::min(80LL * 1024, tile32_lds_budget())) ? 32 : 16;
      const int nblk = R / NT;
      const dim3 grid(xcd_grid(cnt, nblk));
      const size_t lds = static_cast<size_t>(rows) * (NT + 2) * 8 + 16;
      if (NT == 32) {
        if ((e = allow_lds(reinterpret_cast<const void*>(&k_final_synth_mfma<32, PREC>), lds)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_final_synth_mfma<32, PREC>), grid, dim3(256), lds, s, tasks, cnt, nblk, fp, v0, v1, P->d.invD, y, P->l, R);
      } else {
        if ((e = allow_lds(reinterpret_cast<const void*>(&k_final_synth_mfma<16, PREC>), lds)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_final_synth_mfma<16, PREC>), grid, dim3(256), lds, s, tasks, cnt, nblk, fp, v0, v1, P->d.invD, y, P->l, R);
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const long long cnt = P->n_final;
  const double* scale = adjoint ? P->d.invD : P->d.D;
  const double half = adjoint ? 1.0 : 0.5;
  const int NT = 16;
  const int nblk = R / NT;
  const dim3 grid(xcd_grid(cnt, nblk));
  const size_t lds_t = final_trans_lds<16, 128>();
  hipLaunchKernelGGL((k_final_trans_mfma<16, 128, PREC>), grid, dim3(256), lds_t, s,
                     P->d.finals, cnt, nblk, fp, yin, scale, half, v0w, v1w, P->l, R);
  return hipGetLastError();
}

// ------------------------------------------------------------------ batched persistent launch
// Grid-wide barrier for a launch whose work-groups are all resident: arrive with release,
// wait with acquire (agent scope, which writes back / invalidates the L2 of every XCD as
// needed), give up after spin_limit polls and raise *status.  Returns false when the
// launch is to be abandoned.
__device__ bool grid_barrier(unsigned* ctr, unsigned nwg, int* status, long long spin_limit) {
  __shared__ int s_ok;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    long long polls = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < nwg) {
      if (++polls > spin_limit || __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
    if (!ok) __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_ok = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return s_ok != 0;
}

template <int NT, int PREC, bool TRANS>
__device__ void run_item(const BatchItem& it, const BatchGroupDev& g, double* lds) {
  const int t = it.step;
  if (!TRANS) {
    if (it.kind == kItemLevel) {
      const double* in = t == 0 ? nullptr : ((t - 1) % 2 ? g.v1 : g.v0);
      double* out = t % 2 ? g.v1 : g.v0;
      level_synth_body<NT, PREC, false>(g.tasks[it.task], it.blk, g.fp, g.idx, g.pairs, in, out, g.R, g.io, lds);
    } else {
      final_synth_body<NT, PREC, false>(g.finals[it.task], it.blk, g.fp, g.v0, g.v1, g.rowscale, g.y, g.l, g.R, lds);
    }
  } else {
    if (it.kind == kItemLevel) {
      const double* in = t % 2 ? g.v1 : g.v0;
      double* out = t == 0 ? nullptr : ((t - 1) % 2 ? g.v1 : g.v0);
      // the split vectors are read from global memory here: staging them would size every
      // work-group's LDS for the largest pair of output blocks of any group
      level_trans_body<NT, PREC, false, false>(g.tasks[it.task], it.blk, g.fp, g.idx, g.pairs, in, out, g.R, g.io,
                                        lds);
    } else {  // transposed finals always take 16-column blocks, and keep two output tiles per
              // wave and pass (the persistent loop's state leaves no registers for six)
      final_trans_body<16, 128, PREC, false, 2>(g.finals[it.task], it.blk, g.fp, g.y, g.rowscale, g.half, g.v0,
                                                g.v1, g.l, g.R, lds);
    }
  }
}

// Every work-group walks the phases in order; within a phase it takes items from its own
// queue (queue = work-group id mod nq: with nq = 8 the queue of its XCD, since work-groups are
// dealt to the XCDs round-robin) and then from the others, one atomic increment per item.
template <int NT, int PREC, bool TRANS>
__global__ void __launch_bounds__(256, kMinBlocks) k_batch(BatchLaunch bl) {
  extern __shared__ double lds[];
  __shared__ int s_item;
  const int nq = bl.nq;
  const int myq = static_cast<int>(blockIdx.x % nq);
  unsigned* heads = bl.sync;
  unsigned* bars = bl.sync + static_cast<long long>(bl.nphase) * nq;
  for (int ph = 0; ph < bl.nphase; ++ph) {
    for (int d = 0; d < nq; ++d) {
      const int q = (myq + d) % nq;
      const int beg = bl.qoff[ph * nq + q], end = bl.qoff[ph * nq + q + 1];
      if (beg == end) continue;
      for (;;) {
        if (threadIdx.x == 0) s_item = beg + static_cast<int>(atomicAdd(&heads[ph * nq + q], 1u));
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar item loads
        __syncthreads();
        if (i >= end) break;
        const BatchItem it = bl.items[i];
        run_item<NT, PREC, TRANS>(it, bl.groups[it.group], lds);
        __syncthreads();
      }
    }
    if (ph + 1 < bl.nphase && !grid_barrier(&bars[ph], gridDim.x, bl.status, bl.spin_limit)) return;
  }
}

__global__ void k_fill_u32(unsigned* p, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) p[i] = 0u;
}

template <int NT, int PREC, bool TRANS>
const void* batch_fn() {
  return reinterpret_cast<const void*>(&k_batch<NT, PREC, TRANS>);
}

const void* batch_kernel(int nt, int precision, bool trans) {
#define PICK(NT_, P_)                                                             \
  return trans ? batch_fn<NT_, P_, true>() : batch_fn<NT_, P_, false>();
  if (nt == 32) {
    if (precision == SHT_SPLIT32) PICK(32, PSPLIT)
    if (precision == SHT_FP32) PICK(32, P32)
    PICK(32, P64)
  }
  if (precision == SHT_SPLIT32) PICK(16, PSPLIT)
  if (precision == SHT_FP32) PICK(16, P32)
  PICK(16, P64)
#undef PICK
}

}  // namespace

hipError_t transpose_factors(const double* fac, double* fac_t, const FactorBlock* blocks,
                             long long nblocks, hipStream_t s) {
  for (long long b0 = 0; b0 < nblocks; b0 += 1 << 20) {
    const long long nb = std::min<long long>(1 << 20, nblocks - b0);
    hipLaunchKernelGGL(k_transpose_blocks, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, fac,
                       fac_t, blocks + b0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t split_factors(sht_plan_s* P, hipStream_t s) {
  if (P->d.fac_hl) return hipSuccess;
  if (!P->d.fac || !P->d.fac_t) return hipErrorInvalidValue;
  const size_t n = static_cast<size_t>(std::max<long long>(P->n_fac, 4));
  float2* bufs[2] = {nullptr, nullptr};
  for (int b = 0; b < 2; ++b) {
    hipError_t e = dev_alloc(reinterpret_cast<void**>(&bufs[b]), n * sizeof(float2));
    if (e != hipSuccess) {
      if (b) (void)hipFree(bufs[0]);
      return e;
    }
  }
  for (long long b0 = 0; b0 < P->n_blocks; b0 += 1 << 20) {
    const long long nb = std::min<long long>(1 << 20, P->n_blocks - b0);
    hipLaunchKernelGGL(k_split_rows, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, P->d.fac, bufs[0],
                       P->d.blocks + b0, 0);
    hipLaunchKernelGGL(k_split_rows, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, P->d.fac_t,
                       bufs[1], P->d.blocks + b0, 1);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    for (float2* q : bufs) (void)hipFree(q);
    return e;
  }
  P->d.fac_hl = bufs[0];
  P->d.fac_t_hl = bufs[1];
  P->stats.device_bytes += static_cast<long long>(2 * n * sizeof(float2));
  return hipSuccess;
}

bool mfma_ok(int R) { return R % 16 == 0; }

hipError_t launch_level_mfma(const sht_plan_s* P, int step, bool transpose, const double* in,
                             double* out, int R, int precision, hipStream_t s, double* coeff, int only) {
  if (precision == SHT_INT8) return launch_level_i8(P, step, transpose, in, out, R, s, coeff, only);
  CoefIO io{coeff, nullptr,
            P->kind == SHT_COMPLEX ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l, P->l, P->kind};
  for (size_t c = 0; c < P->step_classes[step].size(); ++c) {
    if (only >= 0 && static_cast<int>(c) != only) continue;
    const LaunchClass& lc = P->step_classes[step][c];
    hipError_t e;
    if (precision == SHT_SPLIT32)
      e = level_class<PSPLIT>(P, step, lc, transpose, in, out, R, io, s);
    else if (precision == SHT_FP32)
      e = level_class<P32>(P, step, lc, transpose, in, out, R, io, s);
    else
      e = level_class<P64>(P, step, lc, transpose, in, out, R, io, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_final_mfma(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                             double* v0w, double* v1w, double* y, const double* yin, int R,
                             int precision, bool adjoint, hipStream_t s, int only) {
  if (P->n_final == 0) return hipSuccess;
  if (precision == SHT_INT8) return launch_final_i8(P, transpose, v0, v1, v0w, v1w, y, yin, R, adjoint, s, only);
  if (precision == SHT_SPLIT32)
    return final_launch<PSPLIT>(P, transpose, v0, v1, v0w, v1w, y, yin, R, adjoint, s, only);
  if (precision == SHT_FP32)
    return final_launch<P32>(P, transpose, v0, v1, v0w, v1w, y, yin, R, adjoint, s, only);
  return final_launch<P64>(P, transpose, v0, v1, v0w, v1w, y, yin, R, adjoint, s, only);
}

hipError_t batch_kernel_prepare(int nt, int precision, bool transpose, size_t lds, int* wg_per_cu) {
  if (nt != 16 && nt != 32) return hipErrorInvalidValue;
  const void* fn = batch_kernel(nt, precision, transpose);
  hipError_t e = allow_lds(fn, lds);
  if (e != hipSuccess) return e;
  int n = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 256, lds);
  if (e != hipSuccess) return e;
  *wg_per_cu = n;
  return hipSuccess;
}

hipError_t launch_batch_kernel(int nt, int precision, bool transpose, const BatchLaunch& bl, unsigned grid,
                               size_t lds, hipStream_t s) {
  if (nt != 16 && nt != 32) return hipErrorInvalidValue;
  const void* fn = batch_kernel(nt, precision, transpose);
  BatchLaunch arg = bl;
  void* args[] = {&arg};
  return hipLaunchKernel(fn, dim3(grid), dim3(256), args, lds, s);
}

hipError_t launch_fill_u32(unsigned* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

size_t final_trans_lds_bytes() { return final_trans_lds<16, 128>(); }

}  // namespace sht
