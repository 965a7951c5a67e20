// Butterfly apply on the FP64 matrix cores (v_mfma_f64_16x16x4f64), used when the
// number of R columns is a multiple of 16, i.e. many fields at once.
//
// Each interpolation is a small GEMM with a gathered operand: out = in[skel] + T in[red]
// (synthesis) or in = sum_o scatter(T_o^T w_o, w_o) (transposed).  A work-group takes one
// task and NT columns.  It first stages the task's vector rows for those columns in LDS with
// coalesced loads (all in flight at once), then every wave runs MFMAs on pairs of 16-row
// tiles: the factor fragments (A) stream from global memory in the order the plan packed
// them (a stored column is contiguous, so 16 lanes read 128 consecutive bytes), the vector
// fragments (B) come from LDS through the skeleton / redundant index lists.
//
// Work-groups are numbered so that all column blocks of one task land on the same XCD
// (work-group ids are dealt round-robin over the 8 XCDs): the factor matrix is then read
// from HBM once and served to the other column blocks by that XCD's L2.
//
// MFMA f64 16x16x4 register layout (checked on gfx950): A[i][k] in lane i + 16k, B[k][j]
// in lane j + 16k, and D[4v + lane/16][lane%16] in accumulator element v.
#include <algorithm>

#include "sht_internal.h"

namespace sht {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 zero4() { return d4{0.0, 0.0, 0.0, 0.0}; }

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

// Where a leaf task's vector rows live when they are read from / written to the caller's
// coefficient array directly (the layout change fused into the leaf level).
struct CoefIO {
  double* coeff;  // null: use the internal row buffer instead
  const PairDesc* pairs;
  long long ncoef;
  int l, kind;
};

// Visits the K x NT block of a leaf task (rows j of pair mp starting at column j0; local
// columns c of the NT-column block c0) in an order where consecutive threads touch
// consecutive degrees of one (field, sign): fn(j, c, position or -1 if no such entry).
template <int NT, typename Fn>
__device__ __forceinline__ void for_leaf_block(const CoefIO& io, int mp_m, int mp_p, int j0, int K,
                                               long long c0, Fn&& fn) {
  for (int e = threadIdx.x; e < K * NT; e += 256) {
    const int cc = e & 1;
    const int j = (e >> 1) % K;
    const int g = (e >> 1) / K;  // (field, sign) group for complex, field for real
    const int c = g * 2 + cc;
    const int col = static_cast<int>(c0) + c;
    const int k = mp_m + mp_p + 2 * (j0 + j);
    long long pos;
    if (io.kind == SHT_COMPLEX) {
      const int f = col >> 2, s = (col >> 1) & 1;
      pos = (mp_m == 0 && s == 1) ? -1 : coeff_pos(io.l, SHT_COMPLEX, io.ncoef, f, mp_m, s, k, cc);
    } else {
      const int f = col >> 1;
      pos = (mp_m == 0 && cc == 1) ? -2 : coeff_pos(io.l, SHT_REAL, io.ncoef, f, mp_m, 0, k, cc);
    }
    fn(j, c, pos);
  }
}

// ------------------------------------------------------------------- level, synthesis
template <int NT>
__global__ void __launch_bounds__(256)
k_level_synth_mfma(const LevelTask* __restrict__ tasks, long long ntasks, int nblk,
                   const double* __restrict__ fac, const uint16_t* __restrict__ idx,
                   const double* __restrict__ in, double* __restrict__ out, int R, CoefIO io) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const LevelTask tk = tasks[ti];
  const int K = tk.K;
  const long long c0 = static_cast<long long>(blk) * NT;
  double* xs = lds;                                              // K x LD
  uint16_t* ix = reinterpret_cast<uint16_t*>(lds + K * LD);      // [skel0 red0 skel1 red1]
  const int k0 = tk.k[0], k1 = tk.k[1] < 0 ? 0 : tk.k[1];
  const int nidx = (k0 > 0 ? K : 0) + (k1 > 0 ? K : 0);
  if (io.coeff && tk.mp >= 0) {
    const PairDesc pd = io.pairs[tk.mp];
    const double* cf = io.coeff;
    for_leaf_block<NT>(io, pd.m, pd.p, tk.in_row - pd.in_base, K, c0,
                       [&](int j, int c, long long pos) { xs[j * LD + c] = pos >= 0 ? cf[pos] : 0.0; });
  } else {
    const double* src = in + static_cast<long long>(tk.in_row) * R + c0;
    for (int e = threadIdx.x; e < K * (NT / 2); e += 256) {
      const int row = e / (NT / 2), c2 = e % (NT / 2);
      const double2 v = *reinterpret_cast<const double2*>(src + static_cast<long long>(row) * R + 2 * c2);
      xs[row * LD + 2 * c2] = v.x;
      xs[row * LD + 2 * c2 + 1] = v.y;
    }
  }
  {
    if (k0 > 0)
      for (int e = threadIdx.x; e < K; e += 256) ix[e] = idx[tk.idx[0] + e];
    if (k1 > 0)
      for (int e = threadIdx.x; e < K; e += 256) ix[(k0 > 0 ? K : 0) + e] = idx[tk.idx[1] + e];
  }
  (void)nidx;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lr = lane >> 4;
  const int nm0 = (k0 + 15) >> 4, nm1 = (k1 + 15) >> 4;
  // pairs of row tiles: output 0 tiles, then output 1 tiles
  const int np0 = (nm0 + 1) >> 1, np1 = (nm1 + 1) >> 1;
  for (int q = wave; q < np0 + np1; q += 4) {
    const int o = q < np0 ? 0 : 1;
    const int mt0 = 2 * (o ? q - np0 : q);
    const int k = o ? k1 : k0;
    const int nr = K - k;
    const uint16_t* skel = ix + (o && k0 > 0 ? K : 0);
    const uint16_t* red = skel + k;
    const double* T = fac + tk.fac[o];
    const bool two = mt0 + 1 < (o ? nm1 : nm0);
    d4 acc[2][NTL];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int n = 0; n < NTL; ++n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (mt0 + u) * 16 + 4 * v + lr;
          acc[u][n][v] = row < k ? xs[skel[row] * LD + n * 16 + lc] : 0.0;
        }
      }
    }
    const int i0 = mt0 * 16 + lc, i1 = i0 + 16;
    // factor fragments are fetched PF K-steps ahead (double-buffered in registers) so the
    // global-load latency overlaps the MFMAs of the previous steps
    constexpr int PF = 4;
    const int nsteps = (nr + 3) >> 2;
    double a0c[PF], a1c[PF], a0n[PF], a1n[PF];
    auto fetch = [&](int s0, double* d0, double* d1) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int kk = (s0 + u) * 4 + lr;
        const bool kin = kk < nr;
        const double* Tc = T + static_cast<long long>(kk) * k;
        d0[u] = (kin && i0 < k) ? Tc[i0] : 0.0;
        d1[u] = (kin && two && i1 < k) ? Tc[i1] : 0.0;
      }
    };
    fetch(0, a0c, a1c);
    for (int s0 = 0; s0 < nsteps; s0 += PF) {
      if (s0 + PF < nsteps) fetch(s0 + PF, a0n, a1n);
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int kk = (s0 + u) * 4 + lr;
        const bool kin = kk < nr;
        const double* xr = xs + (kin ? red[kk] : 0) * LD + lc;
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          const double b = kin ? xr[n * 16] : 0.0;
          acc[0][n] = mfma(a0c[u], b, acc[0][n]);
          if (two) acc[1][n] = mfma(a1c[u], b, acc[1][n]);
        }
      }
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        a0c[u] = a0n[u];
        a1c[u] = a1n[u];
      }
    }
    double* ob = out + static_cast<long long>(tk.out_row[o]) * R + c0 + lc;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (mt0 + u) * 16 + 4 * v + lr;
        if (row < k) {
#pragma unroll
          for (int n = 0; n < NTL; ++n) ob[static_cast<long long>(row) * R + n * 16] = acc[u][n][v];
        }
      }
    }
  }
}

// ------------------------------------------------------------------ level, transposed
// LDS holds the accumulated input block (K x NT) and the index lists; the vectors w_o of
// the output blocks are read as B fragments straight from global memory (prefetched with
// the factor fragments).  Output block o contributes T_o^T w_o at rows red_o and w_o at
// rows skel_o (assigned for o = 0, added for o = 1; every row gets exactly one term per
// block).
template <int NT>
__global__ void __launch_bounds__(256)
k_level_trans_mfma(const LevelTask* __restrict__ tasks, long long ntasks, int nblk,
                   const double* __restrict__ fac_t, const uint16_t* __restrict__ idx,
                   const double* __restrict__ win, double* __restrict__ xout, int R, CoefIO io) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const LevelTask tk = tasks[ti];
  const int K = tk.K;
  const long long c0 = static_cast<long long>(blk) * NT;
  const int nouts = tk.k[1] < 0 ? 1 : 2;
  const int k0 = tk.k[0], k1 = tk.k[1] < 0 ? 0 : tk.k[1];
  double* acc_l = lds;
  uint16_t* ix = reinterpret_cast<uint16_t*>(acc_l + K * LD);  // [skel0 red0 skel1 red1]
  for (int o = 0; o < nouts; ++o)
    for (int e = threadIdx.x; e < K; e += 256) ix[o * K + e] = idx[tk.idx[o] + e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lr = lane >> 4;
  for (int o = 0; o < nouts; ++o) {
    const int k = o ? k1 : k0;
    const int nr = K - k;
    const uint16_t* skel = ix + o * K;
    const uint16_t* red = skel + k;
    const double* Tt = fac_t + tk.fac[o];  // nr x k column-major
    const double* wb = win + static_cast<long long>(tk.out_row[o]) * R + c0 + lc;
    const int nm = (nr + 15) >> 4;
    const int np = (nm + 1) >> 1;
    for (int q = wave; q < np; q += 4) {
      const int mt0 = 2 * q;
      const bool two = mt0 + 1 < nm;
      d4 acc[2][NTL];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int n = 0; n < NTL; ++n) acc[u][n] = zero4();
      const int j0 = mt0 * 16 + lc, j1 = j0 + 16;
      constexpr int PF = 4;
      const int nsteps = (k + 3) >> 2;
      double a0c[PF], a1c[PF], a0n[PF], a1n[PF], bc[PF][NTL], bn[PF][NTL];
      auto fetch = [&](int s0, double* d0, double* d1, double (*b)[NTL]) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int i = (s0 + u) * 4 + lr;
          const bool iin = i < k;
          const double* Tr = Tt + static_cast<long long>(i) * nr;
          d0[u] = (iin && j0 < nr) ? Tr[j0] : 0.0;
          d1[u] = (iin && two && j1 < nr) ? Tr[j1] : 0.0;
#pragma unroll
          for (int n = 0; n < NTL; ++n) b[u][n] = iin ? wb[static_cast<long long>(i) * R + n * 16] : 0.0;
        }
      };
      fetch(0, a0c, a1c, bc);
      for (int s0 = 0; s0 < nsteps; s0 += PF) {
        if (s0 + PF < nsteps) fetch(s0 + PF, a0n, a1n, bn);
#pragma unroll
        for (int u = 0; u < PF; ++u) {
#pragma unroll
          for (int n = 0; n < NTL; ++n) {
            acc[0][n] = mfma(a0c[u], bc[u][n], acc[0][n]);
            if (two) acc[1][n] = mfma(a1c[u], bc[u][n], acc[1][n]);
          }
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          a0c[u] = a0n[u];
          a1c[u] = a1n[u];
#pragma unroll
          for (int n = 0; n < NTL; ++n) bc[u][n] = bn[u][n];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = (mt0 + u) * 16 + 4 * v + lr;
          if (j < nr) {
            double* dst = acc_l + static_cast<int>(red[j]) * LD + lc;
#pragma unroll
            for (int n = 0; n < NTL; ++n) {
              if (o == 0)
                dst[n * 16] = acc[u][n][v];
              else
                dst[n * 16] += acc[u][n][v];
            }
          }
        }
      }
    }
    const double* wrow = win + static_cast<long long>(tk.out_row[o]) * R + c0;
    for (int e = threadIdx.x; e < k * NT; e += 256) {
      const int i = e / NT, c = e % NT;
      double* dst = acc_l + static_cast<int>(skel[i]) * LD + c;
      const double val = wrow[static_cast<long long>(i) * R + c];
      if (o == 0)
        *dst = val;
      else
        *dst += val;
    }
    __syncthreads();
  }
  if (io.coeff && tk.mp >= 0) {
    const PairDesc pd = io.pairs[tk.mp];
    double* cf = io.coeff;
    for_leaf_block<NT>(io, pd.m, pd.p, tk.in_row - pd.in_base, K, c0, [&](int j, int c, long long pos) {
      if (pos >= 0)
        cf[pos] = acc_l[j * LD + c];
      else if (pos == -2)  // imaginary part at m = 0 of a real field
        cf[coeff_pos(io.l, SHT_REAL, io.ncoef, static_cast<int>((c0 + c) >> 1), 0, 0,
                     pd.p + 2 * (tk.in_row - pd.in_base + j), 1)] = 0.0;
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
// E = S_0 v_0, O = S_1 v_1 on one pair of 16-row tiles; g(+-x) = (E +- O) / D.
template <int NT>
__global__ void __launch_bounds__(256)
k_final_synth_mfma(const FinalTask* __restrict__ tasks, long long ntasks, int nblk,
                   const double* __restrict__ fac, const double* __restrict__ v0buf,
                   const double* __restrict__ v1buf, const double* __restrict__ invD,
                   double* __restrict__ Y, int l, int R) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  extern __shared__ double lds[];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const FinalTask ft = tasks[ti];
  const long long c0 = static_cast<long long>(blk) * NT;
  const double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1], h = ft.h;
  double* w0 = lds;
  double* w1 = lds + k0 * LD;
  for (int p = 0; p < 2; ++p) {
    const int k = p ? k1 : k0;
    double* w = p ? w1 : w0;
    const double* src = V + static_cast<long long>(ft.in_row[p]) * R + c0;
    for (int e = threadIdx.x; e < k * (NT / 2); e += 256) {
      const int row = e / (NT / 2), c2 = e % (NT / 2);
      const double2 v = *reinterpret_cast<const double2*>(src + static_cast<long long>(row) * R + 2 * c2);
      w[row * LD + 2 * c2] = v.x;
      w[row * LD + 2 * c2 + 1] = v.y;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lr = lane >> 4;
  const double* S0 = fac + ft.fac[0];
  const double* S1 = fac + ft.fac[1];
  const long long ybase = static_cast<long long>(ft.m) * 2 * l;
  const int nm = (h + 15) >> 4;
  for (int mt = wave; mt < nm; mt += 4) {
    d4 E[NTL], O[NTL];
#pragma unroll
    for (int n = 0; n < NTL; ++n) {
      E[n] = zero4();
      O[n] = zero4();
    }
    const int i = mt * 16 + lc;
    const bool iin = i < h;
    // both parities in one prefetched loop: step s < n0 feeds E, the rest feed O
    constexpr int PF = 4;
    const int n0 = (k0 + 3) >> 2, n1 = (k1 + 3) >> 2, nsteps = n0 + n1;
    double ac[PF], an[PF];
    auto fetch = [&](int s0, double* d) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int st = s0 + u;
        const bool odd = st >= n0;
        const int a = (odd ? st - n0 : st) * 4 + lr;
        const bool ain = st < nsteps && a < (odd ? k1 : k0);
        d[u] = (ain && iin) ? (odd ? S1 : S0)[static_cast<long long>(a) * h + i] : 0.0;
      }
    };
    fetch(0, ac);
    for (int s0 = 0; s0 < nsteps; s0 += PF) {
      if (s0 + PF < nsteps) fetch(s0 + PF, an);
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int st = s0 + u;
        if (st >= nsteps) break;
        const bool odd = st >= n0;
        const int a = (odd ? st - n0 : st) * 4 + lr;
        const bool ain = a < (odd ? k1 : k0);
        const double* wr = (odd ? w1 : w0) + (ain ? a : 0) * LD + lc;
        if (!odd) {
#pragma unroll
          for (int n = 0; n < NTL; ++n) E[n] = mfma(ac[u], ain ? wr[n * 16] : 0.0, E[n]);
        } else {
#pragma unroll
          for (int n = 0; n < NTL; ++n) O[n] = mfma(ac[u], ain ? wr[n * 16] : 0.0, O[n]);
        }
      }
#pragma unroll
      for (int u = 0; u < PF; ++u) ac[u] = an[u];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ii = mt * 16 + 4 * v + lr;
      if (ii < h) {
        const int row = ft.row0 + ii;
        const double s = invD[row];
        double* yp = Y + (ybase + l + row) * R + c0 + lc;
        double* ym = Y + (ybase + l - 1 - row) * R + c0 + lc;
#pragma unroll
        for (int n = 0; n < NTL; ++n) {
          yp[n * 16] = (E[n][v] + O[n][v]) * s;
          ym[n * 16] = (E[n][v] - O[n][v]) * s;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ final, transposed
// v_p = S_p^T (half * scale * (G(+x) +- G(-x))): the folded rows are built in LDS chunk by
// chunk; each wave keeps the accumulators of its row tiles across the chunks.
template <int NT, int ICH>
__global__ void __launch_bounds__(256)
k_final_trans_mfma(const FinalTask* __restrict__ tasks, long long ntasks, int nblk,
                   const double* __restrict__ fac_t, const double* __restrict__ Yin,
                   const double* __restrict__ scale, double half, double* __restrict__ v0buf,
                   double* __restrict__ v1buf, int l, int R) {
  constexpr int NTL = NT / 16;
  constexpr int LD = ldp<NT>();
  constexpr int MAXT = 6;  // row tiles per wave (k0 + k1 <= 384)
  __shared__ double eo[2][ICH * LD];
  long long ti;
  int blk;
  if (!xcd_map(ntasks, nblk, ti, blk)) return;
  const FinalTask ft = tasks[ti];
  const long long c0 = static_cast<long long>(blk) * NT;
  double* V = ft.vbuf ? v1buf : v0buf;
  const int k0 = ft.k[0], k1 = ft.k[1], h = ft.h;
  const long long ybase = static_cast<long long>(ft.m) * 2 * l;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lr = lane >> 4;
  const int nm0 = (k0 + 15) >> 4, nm1 = (k1 + 15) >> 4;
  d4 acc[MAXT][NTL];
#pragma unroll
  for (int u = 0; u < MAXT; ++u)
#pragma unroll
    for (int n = 0; n < NTL; ++n) acc[u][n] = zero4();
  for (int i0 = 0; i0 < h; i0 += ICH) {
    const int ih = min(ICH, h - i0);
    __syncthreads();
    for (int e = threadIdx.x; e < ih * NT; e += 256) {
      const int i = e / NT, c = e % NT;
      const int row = ft.row0 + i0 + i;
      const double gp = Yin[(ybase + l + row) * R + c0 + c];
      const double gm = Yin[(ybase + l - 1 - row) * R + c0 + c];
      const double sc = half * scale[row];
      eo[0][i * LD + c] = (gp + gm) * sc;
      eo[1][i * LD + c] = (gp - gm) * sc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
      const int q = wave + 4 * u;  // tile index over [output 0 tiles | output 1 tiles]
      if (q >= nm0 + nm1) break;
      const int p = q < nm0 ? 0 : 1;
      const int k = p ? k1 : k0;
      const int a = (p ? q - nm0 : q) * 16 + lc;
      const double* St = fac_t + ft.fac[p];  // k x h column-major
      const double* src = eo[p];
      constexpr int PF = 4;
      const int nsteps = (ih + 3) >> 2;
      double ac[PF], an[PF];
      auto fetch = [&](int s0, double* d) {
#pragma unroll
        for (int w = 0; w < PF; ++w) {
          const int i = (s0 + w) * 4 + lr;
          d[w] = (i < ih && a < k) ? St[static_cast<long long>(i0 + i) * k + a] : 0.0;
        }
      };
      fetch(0, ac);
      for (int s0 = 0; s0 < nsteps; s0 += PF) {
        if (s0 + PF < nsteps) fetch(s0 + PF, an);
#pragma unroll
        for (int w = 0; w < PF; ++w) {
          const int i = (s0 + w) * 4 + lr;
          const bool iin = i < ih;
          const double* er = src + (iin ? i : 0) * LD + lc;
#pragma unroll
          for (int n = 0; n < NTL; ++n) acc[u][n] = mfma(ac[w], iin ? er[n * 16] : 0.0, acc[u][n]);
        }
#pragma unroll
        for (int w = 0; w < PF; ++w) ac[w] = an[w];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    const int q = wave + 4 * u;
    if (q >= nm0 + nm1) break;
    const int p = q < nm0 ? 0 : 1;
    const int k = p ? k1 : k0;
    const int mt = p ? q - nm0 : q;
    double* vout = V + static_cast<long long>(ft.in_row[p]) * R + c0 + lc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = mt * 16 + 4 * v + lr;
      if (a < k) {
#pragma unroll
        for (int n = 0; n < NTL; ++n) vout[static_cast<long long>(a) * R + n * 16] = acc[u][n][v];
      }
    }
  }
}

__global__ void k_transpose_blocks(const double* __restrict__ fac, double* __restrict__ fac_t,
                                   const FactorBlock* __restrict__ blocks) {
  const FactorBlock b = blocks[blockIdx.x];
  const long long n = static_cast<long long>(b.rows) * b.cols;
  for (long long e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = static_cast<int>(e % b.rows), c = static_cast<int>(e / b.rows);
    fac_t[b.off + static_cast<long long>(r) * b.cols + c] = fac[b.off + e];
  }
}

hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
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

bool mfma_ok(int R) { return R % 16 == 0; }

static hipError_t launch_level_class(const sht_plan_s* P, int step, const LaunchClass& lc,
                                     bool transpose, const double* in, double* out, int R,
                                     const CoefIO& io, hipStream_t s);

hipError_t launch_level_mfma(const sht_plan_s* P, int step, bool transpose, const double* in,
                             double* out, int R, hipStream_t s, double* coeff) {
  CoefIO io{coeff, P->d.pairs,
            P->kind == SHT_COMPLEX ? 4LL * P->l * P->l : 2LL * P->l * P->l + P->l, P->l, P->kind};
  for (const LaunchClass& lc : P->step_classes[step]) {
    hipError_t e = launch_level_class(P, step, lc, transpose, in, out, R, io, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t launch_level_class(const sht_plan_s* P, int step, const LaunchClass& lc,
                                     bool transpose, const double* in, double* out, int R,
                                     const CoefIO& io, hipStream_t s) {
  const long long cnt = lc.cnt;
  if (cnt == 0) return hipSuccess;
  const LevelTask* tasks = P->d.tasks + P->step_off[step] + lc.off;
  const int K = lc.maxK, k = lc.maxk;
  // LDS rows per column: K (the task's input block); use 32 columns while that stays
  // within 100 KiB, else 16.
  (void)k;
  const long long rows = K;
  const int NT = (R % 32 == 0 && rows * 34 * 8 <= 100 * 1024) ? 32 : 16;
  if (rows * 18 * 8 + 4LL * K + 16 > 160 * 1024) return hipErrorInvalidConfiguration;
  const int nblk = R / NT;
  const dim3 grid(xcd_grid(cnt, nblk));
  const int LD = NT + 2;
  hipError_t e;
  if (!transpose) {
    const size_t lds = static_cast<size_t>(K) * LD * 8 + 4 * static_cast<size_t>(K) + 16;
    if (NT == 32) {
      if ((e = allow_lds(reinterpret_cast<const void*>(&k_level_synth_mfma<32>), lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_level_synth_mfma<32>, grid, dim3(256), lds, s, tasks, cnt, nblk, P->d.fac, P->d.idx, in, out, R, io);
    } else {
      if ((e = allow_lds(reinterpret_cast<const void*>(&k_level_synth_mfma<16>), lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_level_synth_mfma<16>, grid, dim3(256), lds, s, tasks, cnt, nblk, P->d.fac, P->d.idx, in, out, R, io);
    }
  } else {
    const size_t lds = static_cast<size_t>(K) * LD * 8 + 4 * static_cast<size_t>(K) + 16;
    if (NT == 32) {
      if ((e = allow_lds(reinterpret_cast<const void*>(&k_level_trans_mfma<32>), lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_level_trans_mfma<32>, grid, dim3(256), lds, s, tasks, cnt, nblk, P->d.fac_t, P->d.idx, in, out, R, io);
    } else {
      if ((e = allow_lds(reinterpret_cast<const void*>(&k_level_trans_mfma<16>), lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_level_trans_mfma<16>, grid, dim3(256), lds, s, tasks, cnt, nblk, P->d.fac_t, P->d.idx, in, out, R, io);
    }
  }
  return hipGetLastError();
}

hipError_t launch_final_mfma(const sht_plan_s* P, bool transpose, const double* v0, const double* v1,
                             double* v0w, double* v1w, double* y, const double* yin, int R,
                             bool adjoint, hipStream_t s) {
  const long long total = P->n_final;
  if (total == 0) return hipSuccess;
  hipError_t e;
  if (!transpose) {
    for (const LaunchClass& lc : P->final_classes) {
      const long long cnt = lc.cnt;
      const FinalTask* tasks = P->d.finals + lc.off;
      const long long rows = 2LL * lc.maxk;
      const int NT = (R % 32 == 0 && rows * 34 * 8 <= 80 * 1024) ? 32 : 16;
      const int nblk = R / NT;
      const dim3 grid(xcd_grid(cnt, nblk));
      const size_t lds = static_cast<size_t>(rows) * (NT + 2) * 8 + 16;
      if (NT == 32) {
        if ((e = allow_lds(reinterpret_cast<const void*>(&k_final_synth_mfma<32>), lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_final_synth_mfma<32>, grid, dim3(256), lds, s, tasks, cnt, nblk, P->d.fac, v0, v1, P->d.invD, y, P->l, R);
      } else {
        if ((e = allow_lds(reinterpret_cast<const void*>(&k_final_synth_mfma<16>), lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_final_synth_mfma<16>, grid, dim3(256), lds, s, tasks, cnt, nblk, P->d.fac, v0, v1, P->d.invD, y, P->l, R);
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  } else {
    const long long cnt = total;
    if (P->final_maxk > 6 * 16 * 4 / 2) return hipErrorInvalidValue;  // k0 + k1 <= 384
    const double* scale = adjoint ? P->d.invD : P->d.D;
    const double half = adjoint ? 1.0 : 0.5;
    const int NT = 16;
    const int nblk = R / NT;
    const dim3 grid(xcd_grid(cnt, nblk));
    hipLaunchKernelGGL((k_final_trans_mfma<16, 128>), grid, dim3(256), 0, s, P->d.finals, cnt, nblk, P->d.fac_t, yin, scale, half, v0w, v1w, P->l, R);
  }
  return hipGetLastError();
}

}  // namespace sht
