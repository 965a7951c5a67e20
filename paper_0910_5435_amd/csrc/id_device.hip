// Interpolative decompositions on the device (Section 3.1 with Lemma interpolation_lemma,
// Remark QR_algorithm and Remark adaptivity), for the butterflies of Section 3.2.
//
// The host builder follows Section 4 literally: one (order, parity) pair at a time, depth
// first, holding only the skeleton columns of unfinished blocks.  This builder keeps the
// whole Q^{(m,p)} of a batch of pairs in HBM instead (at most a few GB per batch; MI355X has
// 288 GB) and runs every block of one level of every pair of the batch at once, one
// work-group per block, level after level.  Each block is the submatrix of its pair's Q on
// the block's rows and on the global columns that the two blocks below it kept as skeletons,
// gathered straight from Q; it is factored exactly as the host does it:
//
//  * Householder QR with column pivoting (largest remaining norm, lowest index on ties),
//    norms downdated after each step and recomputed once cancellation has eaten 6 digits;
//  * the rank is the least k whose trailing block has Frobenius norm <= eps;
//  * T = R11^{-1} R12 by back substitution;
//  * while some |T_ij| > 2, the skeleton column i and redundant column j of the largest one
//    are exchanged and the block refactored without pivoting in the new order (Gu-Eisenstat;
//    taken only if the residual stays within eps, at most 64 times).
//
// The host then assembles the trees from the ranks, column orders and T of every block and
// the final skeleton values S (gathered from Q as well), with the same statistics as the
// depth-first build.  Results agree with the host builder's up to rounding and pivot ties.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <cstring>
#include <vector>

#include "interp_decomp.h"
#include "sht_internal.h"

namespace sht {

namespace {

constexpr int kIdThreads = 512;
constexpr int kIdWaves = kIdThreads / 64;
constexpr int kIdMaxK = 512;     // largest block input length the kernel takes
constexpr int kIdMaxRows = 2048; // largest block height (l <= 2048)

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Sum over the work-group, returned to every thread.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kIdWaves; ++w) s += red[w];
  return s;
}

// Largest value and its lowest index over the work-group (value -1 where a thread has none).
__device__ void block_argmax(double v, int idx, double* redv, int* redi, double& best, int& at) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(idx, o);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    redv[wave] = v;
    redi[wave] = idx;
  }
  __syncthreads();
  best = redv[0];
  at = redi[0];
#pragma unroll
  for (int w = 1; w < kIdWaves; ++w)
    if (redv[w] > best || (redv[w] == best && redi[w] < at)) {
      best = redv[w];
      at = redi[w];
    }
}

struct IdShared {
  double nrm[kIdMaxK], nrm0[kIdMaxK];
  int perm[kIdMaxK], trial[kIdMaxK];
  double tcol[kIdWaves][kIdMaxK];  // one back-substitution column per wave
  double redv[kIdWaves];
  int redi[kIdWaves];
};

// One Householder step at column s of the h x K column-major block M (leading dimension h),
// applied to columns s+1 .. K-1; with norms, their norms are downdated as well.  Every wave
// holds the reflector in registers (RPL rows per lane) and takes columns in turn.  Only R is
// kept: the new diagonal entry goes to M[s][s], the reflector itself is not stored (nothing
// later needs the orthogonal factor).
template <int RPL>
__device__ void householder(double* M, int h, int K, int s, IdShared& sh, bool norms) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* col = M + static_cast<long long>(s) * h;
  const double alpha = col[s];
  double v[RPL];
  double x2 = 0.0;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = s + 1 + lane + 64 * u;
    v[u] = i < h ? col[i] : 0.0;
    x2 += v[u] * v[u];
  }
  const double xn2 = wave_sum(x2);  // the same in every wave
  const bool reflect = xn2 > 0.0;   // else the column is already triangular: H = I
  double tau = 0.0;
  if (reflect) {
    const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    tau = (beta - alpha) / beta;
    const double scale = 1.0 / (alpha - beta);
#pragma unroll
    for (int u = 0; u < RPL; ++u) v[u] *= scale;
  }
  for (int j = s + 1 + wave; j < K; j += kIdWaves) {
    double* cj = M + static_cast<long long>(j) * h;
    double c[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int i = s + 1 + lane + 64 * u;
      c[u] = i < h ? cj[i] : 0.0;
    }
    double cjs = cj[s];
    double sq = 0.0;
    if (reflect) {
      double dot = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) dot += v[u] * c[u];
      dot = wave_sum(dot);
      const double d = tau * (cjs + dot);
      cjs -= d;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int i = s + 1 + lane + 64 * u;
        c[u] -= d * v[u];
        if (i < h) cj[i] = c[u];
        sq += c[u] * c[u];
      }
      if (lane == 0) cj[s] = cjs;
    } else {
#pragma unroll
      for (int u = 0; u < RPL; ++u) sq += c[u] * c[u];
    }
    if (norms) {
      double nv = sh.nrm[j] - cjs * cjs;
      if (nv < 1e-6 * sh.nrm0[j]) {  // cancellation: recompute from the trailing rows
        nv = wave_sum(sq);
        if (lane == 0) sh.nrm0[j] = nv;
      }
      if (lane == 0) sh.nrm[j] = nv;
    }
  }
  __syncthreads();
  // every wave has read alpha by now; the next barrier (a reduction of the next step, or the
  // one before the back substitution) publishes the new diagonal entry
  if (reflect && threadIdx.x == 0) M[static_cast<long long>(s) * h + s] = -copysign(sqrt(alpha * alpha + xn2), alpha);
}

// Copies columns src[order[c]] (rows [row0, row0 + h) of the pair's Q) into M.
__device__ void gather_block(const double* __restrict__ q, int ldq, int row0, int h, int K,
                             const int* __restrict__ gc, const int* order, double* M) {
  const long long n = static_cast<long long>(h) * K;
  for (long long e = threadIdx.x; e < n; e += kIdThreads) {
    const int c = static_cast<int>(e / h), i = static_cast<int>(e % h);
    M[e] = q[static_cast<long long>(gc[order[c]]) * ldq + row0 + i];
  }
  __syncthreads();
}

// T = R11^{-1} R12 (k x (K - k), column-major) into t; returns max |T| to every thread.
__device__ double solve_t(const double* M, int h, int K, int k, double* t, IdShared& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mx = 0.0;
  double* tl = sh.tcol[wave];
  for (int j = wave; j < K - k; j += kIdWaves) {
    const double* rj = M + static_cast<long long>(k + j) * h;
    for (int r = lane; r < k; r += 64) tl[r] = rj[r];
    __builtin_amdgcn_wave_barrier();
    for (int i = k - 1; i >= 0; --i) {
      const double* ri = M + static_cast<long long>(i) * h;
      const double ti = tl[i] / ri[i];
      mx = fmax(mx, fabs(ti));
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) tl[i] = ti;
      for (int r = lane; r < i; r += 64) tl[r] -= ti * ri[r];
      __builtin_amdgcn_wave_barrier();
    }
    double* tj = t + static_cast<long long>(j) * k;
    for (int r = lane; r < k; r += 64) tj[r] = tl[r];
    __builtin_amdgcn_wave_barrier();
  }
  mx = wave_max(mx);
  __syncthreads();
  if (lane == 0) sh.redv[wave] = mx;
  __syncthreads();
  double out = 0.0;
#pragma unroll
  for (int w = 0; w < kIdWaves; ++w) out = fmax(out, sh.redv[w]);
  __syncthreads();
  return out;
}

template <int RPL>
__global__ void __launch_bounds__(kIdThreads)
k_id_blocks(const double* __restrict__ Q, int ldq, const IdBlockDesc* __restrict__ blocks, const int* __restrict__ gcols,
            double* __restrict__ work, double* __restrict__ tpool, int* __restrict__ perm_out,
            int* __restrict__ k_out, double* __restrict__ maxt_out, double eps2) {
  __shared__ IdShared sh;
  const IdBlockDesc bd = blocks[blockIdx.x];
  const int h = bd.h, K = bd.K, row0 = bd.row0;
  const double* q = Q + bd.q;
  const int* gc = gcols + bd.gcols;
  double* M = work + bd.work;
  double* T = tpool + bd.tslot;
  for (int c = threadIdx.x; c < K; c += kIdThreads) sh.perm[c] = c;
  __syncthreads();
  gather_block(q, ldq, row0, h, K, gc, sh.perm, M);
  // column norms, one wave per column
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < K; j += kIdWaves) {
      const double* cj = M + static_cast<long long>(j) * h;
      double s = 0.0;
      for (int i = lane; i < h; i += 64) s += cj[i] * cj[i];
      s = wave_sum(s);
      if (lane == 0) sh.nrm[j] = sh.nrm0[j] = s;
    }
  }
  __syncthreads();
  const int kmax = min(h, K);
  int s = 0;
  for (; s < kmax; ++s) {
    double part = 0.0, best = -1.0;
    int at = K;
    for (int j = s + threadIdx.x; j < K; j += kIdThreads) {
      const double v = sh.nrm[j];
      part += v;
      if (v > best) {  // increasing j per thread: the first of equal values wins
        best = v;
        at = j;
      }
    }
    const double resid = block_sum(part, sh.redv);
    if (resid <= eps2) break;
    int p;
    double pv;
    block_argmax(best, at, sh.redv, sh.redi, pv, p);
    if (p != s) {
      double* cs = M + static_cast<long long>(s) * h;
      double* cp = M + static_cast<long long>(p) * h;
      for (int i = threadIdx.x; i < h; i += kIdThreads) {
        const double a = cs[i];
        cs[i] = cp[i];
        cp[i] = a;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const int tp = sh.perm[s];
        sh.perm[s] = sh.perm[p];
        sh.perm[p] = tp;
        double tv = sh.nrm[s];
        sh.nrm[s] = sh.nrm[p];
        sh.nrm[p] = tv;
        tv = sh.nrm0[s];
        sh.nrm0[s] = sh.nrm0[p];
        sh.nrm0[p] = tv;
      }
    }
    __syncthreads();
    householder<RPL>(M, h, K, s, sh, true);
    if (threadIdx.x == 0) sh.nrm[s] = 0.0;
    __syncthreads();
  }
  const int k = s;
  double mt = solve_t(M, h, K, k, T, sh);
  // Gu-Eisenstat exchanges while an interpolation coefficient exceeds 2
  for (int it = 0; it < 64 && k > 0 && k < K && mt > 2.0; ++it) {
    const int nt = k * (K - k);
    double best = -1.0;
    int at = nt;
    for (int e = threadIdx.x; e < nt; e += kIdThreads) {
      const double v = fabs(T[e]);
      if (v > best) {
        best = v;
        at = e;
      }
    }
    double bv;
    int arg;
    block_argmax(best, at, sh.redv, sh.redi, bv, arg);
    const int i = arg % k, j = arg / k;
    for (int c = threadIdx.x; c < K; c += kIdThreads) sh.trial[c] = sh.perm[c];
    __syncthreads();
    if (threadIdx.x == 0) {
      const int a = sh.trial[i];
      sh.trial[i] = sh.trial[k + j];
      sh.trial[k + j] = a;
    }
    __syncthreads();
    gather_block(q, ldq, row0, h, K, gc, sh.trial, M);
    for (int qq = 0; qq < k; ++qq) householder<RPL>(M, h, K, qq, sh, false);
    double part = 0.0;
    for (long long e = threadIdx.x; e < static_cast<long long>(K - k) * (h - k); e += kIdThreads) {
      const int c = k + static_cast<int>(e / (h - k)), r = k + static_cast<int>(e % (h - k));
      const double v = M[static_cast<long long>(c) * h + r];
      part += v * v;
    }
    const double resid = block_sum(part, sh.redv);
    if (resid > eps2) break;  // T still holds the accepted factorization's coefficients
    for (int c = threadIdx.x; c < K; c += kIdThreads) sh.perm[c] = sh.trial[c];
    __syncthreads();
    mt = solve_t(M, h, K, k, T, sh);
  }
  for (int c = threadIdx.x; c < K; c += kIdThreads) perm_out[bd.gcols + c] = sh.perm[c];
  if (threadIdx.x == 0) {
    k_out[blockIdx.x] = k;
    maxt_out[blockIdx.x] = mt;
  }
}

// Chunk `chunk` of the column generator (npairs x C x l) into the pairs' full matrices.
__global__ void k_place_chunk(const double* __restrict__ chunk_buf, double* __restrict__ Q,
                              const long long* __restrict__ qoff, const int* __restrict__ ncols, int C, int l,
                              int chunk) {
  const int b = blockIdx.y;
  const int w = min(C, ncols[b] - chunk * C);
  if (w <= 0) return;
  const long long n = static_cast<long long>(w) * l;
  const double* src = chunk_buf + static_cast<long long>(b) * C * l;
  double* dst = Q + qoff[b] + static_cast<long long>(chunk) * C * l;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += gridDim.x * 256LL) dst[e] = src[e];
}

// Packed copies: item i moves len[i] doubles from src[soff[i]] to dst[doff[i]] (T compaction),
// or, with gather, the h x k final skeleton S from Q (rows row0.., columns listed at cols).
struct CopyItem {
  long long src, dst;
  int len;      // doubles (copy) or h (gather)
  int k;        // gather: columns
  int row0;     // gather: first row
  long long cols;  // gather: offset of the k global columns
};

__global__ void k_copy_items(const double* __restrict__ src, double* __restrict__ dst, const CopyItem* __restrict__ items,
                             const int* __restrict__ cols, int ldq, int gather) {
  const CopyItem it = items[blockIdx.x];
  if (!gather) {
    for (int e = threadIdx.x; e < it.len; e += 256) dst[it.dst + e] = src[it.src + e];
    return;
  }
  const long long n = static_cast<long long>(it.len) * it.k;
  for (long long e = threadIdx.x; e < n; e += 256) {
    const int a = static_cast<int>(e / it.len), i = static_cast<int>(e % it.len);
    dst[it.dst + e] = src[it.src + static_cast<long long>(cols[it.cols + a]) * ldq + it.row0 + i];
  }
}

// A device buffer that grows on demand (contents not kept).
struct Grow {
  void* p = nullptr;
  size_t cap = 0;
  ~Grow() {
    if (p) (void)hipFree(p);
  }
  hipError_t fit(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    const hipError_t e = dev_alloc(&p, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) cap = bytes;
    return e;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// fn(i) for i in [0, n) on the host threads.
template <typename F>
void par_for(int n, F&& fn) {
  const int nt = std::max(1, std::min(host_thread_count(), n / 64 + 1));
  if (nt == 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int i = next++; i < n; i = next++) fn(i);
    });
  for (auto& x : th) x.join();
}

// Pinned host memory that grows on demand (contents not kept).
struct Pinned {
  void* p = nullptr;
  size_t cap = 0;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t fit(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const hipError_t e = pinned_alloc(&p, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) cap = bytes;
    return e;
  }
  double* d() const { return static_cast<double*>(p); }
};

// Streams and events of the builder, released on every exit path.
struct Sync {
  hipStream_t cs = nullptr, xs = nullptr;  // compute, copies of T to the host
  hipEvent_t packed[2] = {nullptr, nullptr}, copied[2] = {nullptr, nullptr};
  ~Sync() {
    if (cs) (void)hipStreamSynchronize(cs);
    if (xs) (void)hipStreamSynchronize(xs);
    for (int i = 0; i < 2; ++i) {
      if (packed[i]) (void)hipEventDestroy(packed[i]);
      if (copied[i]) (void)hipEventDestroy(copied[i]);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (xs) (void)hipStreamDestroy(xs);
  }
  hipError_t init() {
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&xs, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipEventCreateWithFlags(&packed[i], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&copied[i], hipEventDisableTiming);
    }
    return e;
  }
};

// The T of one level waiting on its way to the host: where each block's T sits in the pinned
// buffer, and which IdResult takes it.
struct PendingT {
  int slot = -1;
  std::vector<IdResult*> res;
  std::vector<long long> at;
  std::vector<int> len;
};

struct HostBlock {
  int b, t, r, c;          // batch pair, level, row node, column node
  int row0, h, K;
  std::vector<int> gcols;  // global columns of the input
};

}  // namespace

#define DEV_TRY(expr)                                              \
  do {                                                             \
    const hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return _e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EHIP; \
  } while (0)

int build_trees_on_device(sht_plan_s* P, std::vector<BfTree>& trees, int first_pair, CacheAppend append,
                          double& t_cols, double& t_comp) {
  const int l = P->l, C = P->C;
  const int npairs = static_cast<int>(trees.size());
  const double eps2 = P->eps * P->eps;
  for (int mp = first_pair; mp < npairs; ++mp)
    if (static_cast<long long>(2) * C > kIdMaxK && P->levels[mp] > 0) return SHT_EUNSUPPORTED;
  if (C > kIdMaxK) return SHT_EUNSUPPORTED;
  // nodes and the column generator's state
  std::vector<double> sw(l);
  for (int i = 0; i < l; ++i) sw[i] = std::sqrt(2.0 * P->wp[i]);
  Grow dx, dsw, dm, dp, dn, dprev, dcur, dexp, dchunk, dQ, dqoff, dwork, dT, dperm, dk, dmt, ddesc, dgc, ditems, dS;
  Grow dcomp[2];
  Pinned hT[2];
  Sync sy;
  DEV_TRY(sy.init());
  const hipStream_t cs = sy.cs;
  // copies the waiting T of a level into its IdResults (after its copy to the host is done)
  auto finish = [&](PendingT& pt) -> int {
    if (pt.slot < 0) return SHT_OK;
    if (hipEventSynchronize(sy.copied[pt.slot]) != hipSuccess) return SHT_EHIP;
    const double* src = hT[pt.slot].d();
    par_for(static_cast<int>(pt.res.size()), [&](int u) { pt.res[u]->T.assign(src + pt.at[u], src + pt.at[u] + pt.len[u]); });
    pt = PendingT{};
    return SHT_OK;
  };
  DEV_TRY(dx.fit(8 * l));
  DEV_TRY(dsw.fit(8 * l));
  DEV_TRY(hipMemcpy(dx.p, P->xp.data(), 8 * l, hipMemcpyHostToDevice));
  DEV_TRY(hipMemcpy(dsw.p, sw.data(), 8 * l, hipMemcpyHostToDevice));
  // batches of pairs whose full matrices take about 4 GiB
  const size_t budget = size_t(4) << 30;
  int b0 = first_pair;
  while (b0 < npairs) {
    int nb = 0;
    size_t qbytes = 0;
    while (b0 + nb < npairs) {
      const size_t qb = static_cast<size_t>(l) * std::max(1, P->n_cols[b0 + nb]) * 8;
      if (nb > 0 && qbytes + qb > budget) break;
      qbytes += qb;
      ++nb;
    }
    double ta = now_s();
    std::vector<int> hm(nb), hp(nb), hn(nb);
    std::vector<long long> qoff(nb);
    long long qo = 0;
    int leaves = 1, Lmax = 0;
    for (int b = 0; b < nb; ++b) {
      const int mp = b0 + b;
      hm[b] = mp / 2;
      hp[b] = mp % 2;
      hn[b] = P->n_cols[mp];
      qoff[b] = qo;
      qo += static_cast<long long>(l) * std::max(1, hn[b]);
      leaves = std::max(leaves, 1 << P->levels[mp]);
      Lmax = std::max(Lmax, P->levels[mp]);
      trees[mp].init(l, hn[b], C, P->levels[mp], P->eps);
    }
    DEV_TRY(dm.fit(4 * nb));
    DEV_TRY(dp.fit(4 * nb));
    DEV_TRY(dn.fit(4 * nb));
    DEV_TRY(dprev.fit(16 * static_cast<size_t>(nb) * l));
    DEV_TRY(dcur.fit(16 * static_cast<size_t>(nb) * l));
    DEV_TRY(dexp.fit(4 * static_cast<size_t>(nb) * l));
    DEV_TRY(dchunk.fit(8 * static_cast<size_t>(nb) * C * l));
    DEV_TRY(dQ.fit(8 * static_cast<size_t>(qo)));
    DEV_TRY(dqoff.fit(8 * static_cast<size_t>(nb)));
    DEV_TRY(hipMemcpyAsync(dm.p, hm.data(), 4 * nb, hipMemcpyHostToDevice, cs));
    DEV_TRY(hipMemcpyAsync(dp.p, hp.data(), 4 * nb, hipMemcpyHostToDevice, cs));
    DEV_TRY(hipMemcpyAsync(dn.p, hn.data(), 4 * nb, hipMemcpyHostToDevice, cs));
    DEV_TRY(hipMemcpyAsync(dqoff.p, qoff.data(), 8 * nb, hipMemcpyHostToDevice, cs));
    ColumnBatch cb;
    cb.npairs = nb;
    cb.l = l;
    cb.C = C;
    cb.d_m = dm.as<int>();
    cb.d_p = dp.as<int>();
    cb.d_ncols = dn.as<int>();
    cb.d_prev = dprev.as<double>();
    cb.d_cur = dcur.as<double>();
    cb.d_exp = dexp.as<int>();
    cb.d_out = dchunk.as<double>();
    cb.d_x = dx.as<double>();
    cb.d_sw = dsw.as<double>();
    DEV_TRY(legendre_seed(cb, cs));
    for (int c = 0; c < leaves; ++c) {
      DEV_TRY(legendre_chunk(cb, c, cs));
      hipLaunchKernelGGL(k_place_chunk, dim3(std::max(1, std::min(64, (C * l + 255) / 256)), nb), dim3(256), 0,
                         cs, dchunk.as<double>(), dQ.as<double>(), dqoff.as<long long>(), dn.as<int>(), C, l, c);
      DEV_TRY(hipGetLastError());
    }
    DEV_TRY(hipStreamSynchronize(cs));
    const double tb = now_s();
    t_cols += tb - ta;

    // ids[b][t][r * ncol + c], and the global skeleton columns of every block
    std::vector<std::vector<std::vector<IdResult>>> ids(nb);
    std::vector<std::vector<std::vector<std::vector<int>>>> skg(nb);
    for (int b = 0; b < nb; ++b) {
      const BfTree& tr = trees[b0 + b];
      ids[b].resize(tr.L() + 1);
      skg[b].resize(tr.L() + 1);
      for (int t = 0; t <= tr.L(); ++t) {
        ids[b][t].resize(static_cast<size_t>(tr.nrow(t)) * tr.ncol(t));
        skg[b][t].resize(ids[b][t].size());
      }
    }
    PendingT pend;
    for (int t = 0; t <= Lmax; ++t) {
      std::vector<HostBlock> hb;
      for (int b = 0; b < nb; ++b) {
        const BfTree& tr = trees[b0 + b];
        if (tr.L() < t) continue;
        if (t == 0) {
          for (int c = 0; c < tr.ncol(0); ++c) {
            HostBlock x{b, 0, 0, c, 0, l, tr.leaf_width(c), {}};
            for (int j = 0; j < x.K; ++j) x.gcols.push_back(c * C + j);
            hb.push_back(std::move(x));
          }
          continue;
        }
        const int ncp = tr.ncol(t - 1);
        for (int qn = 0; qn < tr.nrow(t - 1); ++qn)
          for (int cc = 0; cc < tr.ncol(t); ++cc) {
            std::vector<int> g = skg[b][t - 1][qn * ncp + 2 * cc];
            const std::vector<int>& gr = skg[b][t - 1][qn * ncp + 2 * cc + 1];
            g.insert(g.end(), gr.begin(), gr.end());
            for (int half = 0; half < 2; ++half) {
              const int r = 2 * qn + half;
              hb.push_back({b, t, r, cc, tr.row_lo(t, r), tr.row_h(t, r), static_cast<int>(g.size()), g});
            }
          }
      }
      // blocks with nothing to factor are settled here (as interp_decomp settles them)
      std::vector<int> dev;
      for (int i = 0; i < static_cast<int>(hb.size()); ++i) {
        const HostBlock& x = hb[i];
        IdResult& res = ids[x.b][x.t][x.r * trees[b0 + x.b].ncol(x.t) + x.c];
        if (x.K == 0 || x.h == 0) {
          res = IdResult{};
          for (int j = 0; j < x.K; ++j) res.red.push_back(j);
          continue;
        }
        if (x.K > kIdMaxK) return SHT_EUNSUPPORTED;
        dev.push_back(i);
      }
      const int nd = static_cast<int>(dev.size());
      if (nd > 0) {
        std::vector<IdBlockDesc> desc(nd);
        std::vector<int> gpool;
        long long wo = 0, to = 0;
        for (int u = 0; u < nd; ++u) {
          const HostBlock& x = hb[dev[u]];
          IdBlockDesc& d = desc[u];
          d.q = qoff[x.b];
          d.gcols = static_cast<long long>(gpool.size());
          d.work = wo;
          d.tslot = to;
          d.row0 = x.row0;
          d.h = x.h;
          d.K = x.K;
          gpool.insert(gpool.end(), x.gcols.begin(), x.gcols.end());
          wo += static_cast<long long>(x.h) * x.K;
          to += static_cast<long long>(x.K) * x.K / 4 + 1;
        }
        DEV_TRY(ddesc.fit(sizeof(IdBlockDesc) * nd));
        DEV_TRY(dgc.fit(4 * gpool.size()));
        DEV_TRY(dperm.fit(4 * gpool.size()));
        DEV_TRY(dwork.fit(8 * static_cast<size_t>(wo)));
        DEV_TRY(dT.fit(8 * static_cast<size_t>(to)));
        DEV_TRY(dk.fit(4 * nd));
        DEV_TRY(dmt.fit(8 * nd));
        DEV_TRY(hipMemcpyAsync(ddesc.p, desc.data(), sizeof(IdBlockDesc) * nd, hipMemcpyHostToDevice, cs));
        DEV_TRY(hipMemcpyAsync(dgc.p, gpool.data(), 4 * gpool.size(), hipMemcpyHostToDevice, cs));
        int maxh = 1;
        for (const IdBlockDesc& d : desc) maxh = std::max(maxh, d.h);
        if (maxh > kIdMaxRows) return SHT_EUNSUPPORTED;
#define ID_LAUNCH(RPLV)                                                                                \
  hipLaunchKernelGGL(k_id_blocks<RPLV>, dim3(nd), dim3(kIdThreads), 0, cs, dQ.as<double>(), l,             \
                     ddesc.as<IdBlockDesc>(), dgc.as<int>(), dwork.as<double>(), dT.as<double>(), dperm.as<int>(), \
                     dk.as<int>(), dmt.as<double>(), eps2)
        const int rpl = (maxh + 62) / 64;  // rows below the diagonal per lane
        if (rpl <= 1)
          ID_LAUNCH(1);
        else if (rpl <= 2)
          ID_LAUNCH(2);
        else if (rpl <= 4)
          ID_LAUNCH(4);
        else if (rpl <= 8)
          ID_LAUNCH(8);
        else if (rpl <= 16)
          ID_LAUNCH(16);
        else
          ID_LAUNCH(32);
#undef ID_LAUNCH
        DEV_TRY(hipGetLastError());
        // the previous level's T reaches its IdResults while this level is factored
        if (const int rc = finish(pend)) return rc;
        std::vector<int> kk(nd), perm(gpool.size());
        std::vector<double> mt(nd);
        DEV_TRY(hipMemcpyAsync(kk.data(), dk.p, 4 * nd, hipMemcpyDeviceToHost, cs));
        DEV_TRY(hipMemcpyAsync(mt.data(), dmt.p, 8 * nd, hipMemcpyDeviceToHost, cs));
        DEV_TRY(hipMemcpyAsync(perm.data(), dperm.p, 4 * perm.size(), hipMemcpyDeviceToHost, cs));
        DEV_TRY(hipStreamSynchronize(cs));
        // T of every block, packed
        std::vector<CopyItem> items(nd);
        long long co = 0;
        for (int u = 0; u < nd; ++u) {
          const int K = desc[u].K, k = kk[u];
          if (k < 0 || k > std::min(desc[u].h, K)) return SHT_EINTERNAL;
          items[u] = CopyItem{desc[u].tslot, co, k * (K - k), 0, 0, 0};
          co += static_cast<long long>(k) * (K - k);
        }
        // pack the level's T on the device, then copy it to pinned memory on the copy stream
        const int slot = t % 2;
        if (co > 0) {
          DEV_TRY(dcomp[slot].fit(8 * static_cast<size_t>(co)));
          DEV_TRY(hT[slot].fit(8 * static_cast<size_t>(co)));
          DEV_TRY(ditems.fit(sizeof(CopyItem) * nd));
          DEV_TRY(hipMemcpyAsync(ditems.p, items.data(), sizeof(CopyItem) * nd, hipMemcpyHostToDevice, cs));
          hipLaunchKernelGGL(k_copy_items, dim3(nd), dim3(256), 0, cs, dT.as<double>(), dcomp[slot].as<double>(),
                             ditems.as<CopyItem>(), nullptr, 0, 0);
          DEV_TRY(hipGetLastError());
          DEV_TRY(hipEventRecord(sy.packed[slot], cs));
          DEV_TRY(hipStreamWaitEvent(sy.xs, sy.packed[slot], 0));
          DEV_TRY(hipMemcpyAsync(hT[slot].p, dcomp[slot].p, 8 * static_cast<size_t>(co), hipMemcpyDeviceToHost, sy.xs));
          DEV_TRY(hipEventRecord(sy.copied[slot], sy.xs));
          // the items upload above reads `items` from pageable memory: keep it until the copy
          DEV_TRY(hipStreamSynchronize(cs));
          pend.slot = slot;
          pend.res.assign(nd, nullptr);
          pend.at.assign(nd, 0);
          pend.len.assign(nd, 0);
        }
        par_for(nd, [&](int u) {
          const HostBlock& x = hb[dev[u]];
          const int K = x.K, k = kk[u];
          const int* pr = perm.data() + desc[u].gcols;
          const size_t slot = static_cast<size_t>(x.r) * trees[b0 + x.b].ncol(x.t) + x.c;
          IdResult& res = ids[x.b][x.t][slot];
          res.k = k;
          res.skel.assign(pr, pr + k);
          res.red.assign(pr + k, pr + K);
          res.T.clear();
          if (co > 0) {
            pend.res[u] = &res;
            pend.at[u] = items[u].dst;
            pend.len[u] = items[u].len;
          }
          res.max_abs_t = mt[u];
          std::vector<int>& sg = skg[x.b][x.t][slot];
          sg.resize(k);
          for (int a = 0; a < k; ++a) sg[a] = x.gcols[pr[a]];
        });
      }
      for (const HostBlock& x : hb)  // settled blocks keep no skeleton
        if (x.K == 0 || x.h == 0) skg[x.b][x.t][x.r * trees[b0 + x.b].ncol(x.t) + x.c].clear();
    }
    if (const int rc = finish(pend)) return rc;
    // final skeletons S = Q[rows of node r at level L, skeleton columns of block (L, r, 0)]
    std::vector<CopyItem> fitems;
    std::vector<int> fcols;
    long long fo = 0;
    for (int b = 0; b < nb; ++b) {
      const BfTree& tr = trees[b0 + b];
      const int L = tr.L();
      for (int r = 0; r < tr.nrow(L); ++r) {
        const std::vector<int>& g = skg[b][L][r];
        const int h = tr.row_h(L, r), k = static_cast<int>(g.size());
        fitems.push_back(CopyItem{qoff[b], fo, h, k, tr.row_lo(L, r), static_cast<long long>(fcols.size())});
        fcols.insert(fcols.end(), g.begin(), g.end());
        fo += static_cast<long long>(h) * k;
      }
    }
    if (fo > 0) {
      DEV_TRY(dS.fit(8 * static_cast<size_t>(fo)));
      DEV_TRY(hT[0].fit(8 * static_cast<size_t>(fo)));
      DEV_TRY(ditems.fit(sizeof(CopyItem) * fitems.size()));
      DEV_TRY(dgc.fit(4 * std::max<size_t>(1, fcols.size())));
      DEV_TRY(hipMemcpyAsync(ditems.p, fitems.data(), sizeof(CopyItem) * fitems.size(), hipMemcpyHostToDevice, cs));
      DEV_TRY(hipMemcpyAsync(dgc.p, fcols.data(), 4 * fcols.size(), hipMemcpyHostToDevice, cs));
      hipLaunchKernelGGL(k_copy_items, dim3(static_cast<unsigned>(fitems.size())), dim3(256), 0, cs,
                         dQ.as<double>(), dS.as<double>(), ditems.as<CopyItem>(), dgc.as<int>(), l, 1);
      DEV_TRY(hipGetLastError());
      DEV_TRY(hipMemcpyAsync(hT[0].p, dS.p, 8 * static_cast<size_t>(fo), hipMemcpyDeviceToHost, cs));
      DEV_TRY(hipStreamSynchronize(cs));
    }
    const double* sall = hT[0].d();
    std::vector<size_t> ffirst(nb + 1, 0);
    for (int b = 0; b < nb; ++b) ffirst[b + 1] = ffirst[b] + trees[b0 + b].nrow(trees[b0 + b].L());
    std::atomic<int> bad{0};
    par_for(nb, [&](int b) {
      BfTree& tr = trees[b0 + b];
      const int L = tr.L();
      std::vector<std::vector<double>> S(tr.nrow(L));
      std::vector<std::vector<int>> cols(tr.nrow(L));
      for (int r = 0; r < tr.nrow(L); ++r) {
        const CopyItem& it = fitems[ffirst[b] + r];
        S[r].assign(sall + it.dst, sall + it.dst + static_cast<long long>(it.len) * it.k);
        cols[r] = std::move(skg[b][L][r]);
      }
      try {
        tr.assemble(ids[b], S, cols);
      } catch (...) {
        bad = SHT_EINTERNAL;
      }
    });
    if (bad) return bad;
    t_comp += now_s() - tb;
    if (append) {
      const int rc = append(b0, b0 + nb);
      if (rc != SHT_OK) return rc;
    }
    b0 += nb;
  }
  return SHT_OK;
}

}  // namespace sht
