// K-means++ over the feature columns of a binary X (the paper's K-means++
// subsection; Euclidean distance), on the GPU in exact integer arithmetic.
//
// Seeding: the first centre is draw_0 mod F; each further centre j is the
// smallest feature whose inclusive prefix sum of D^2 exceeds draw_i mod T,
// with D^2_j = min over chosen centres c of c_j + c_c - 2 (X^T X)_{jc} and
// T = sum_j D^2_j.  A Gram column X^T x_c is one CSC pass over an indicator.
//
// Lloyd: a cluster s is its member set (initially its centre); with
// S_s = sum of member columns, n_s = |members|, Q_s = ||S_s||^2 and
// h_js = x_j^T S_s, feature j moves to the lowest s minimising the rational
// (Q_s - 2 n_s h_js) / n_s^2 (compared exactly with 128-bit products).
// h_j. is a histogram over the clusters of the features that share a row
// with j; only touched clusters and s0 = argmin_s Q_s / n_s^2 can win.
// Empty clusters drop out; survivors are renumbered in increasing order.
#include <climits>

#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "rr_device.h"

namespace rr {

// ----------------------------------------------------------------------------
// seeding
// ----------------------------------------------------------------------------
constexpr int kSeedChunk = 1024;   // features per block in the D^2 sums

struct SeedState {
  long long r_rem;   // remaining draw inside the selected chunk
  int chunk;         // selected chunk
  int stop;          // 1 once T = 0 (every feature coincides with a centre)
  int n_centres;
  int pad;
};

__global__ void k_seed_first(const unsigned long long* draws, int F, int* centres,
                             SeedState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    centres[0] = (int)(draws[0] % (unsigned long long)F);
    st->stop = 0;
    st->n_centres = 1;
  }
}

// ind[rows of column centres[slot_prev]] = 0, then ind[rows of centres[slot]] = 1
__global__ void k_indicator(const int* __restrict__ col_ptr, const int* __restrict__ row_idx,
                            const int* centres, const int* __restrict__ finv, int slot,
                            double value, double* ind, const SeedState* st) {
  if (st->stop) return;
  const int c = finv[centres[slot]];
  const int a = col_ptr[c], b = col_ptr[c + 1];
  for (int e = a + blockIdx.x * blockDim.x + threadIdx.x; e < b; e += gridDim.x * blockDim.x)
    ind[row_idx[e]] = value;
}

// d2 = min(d2, c_j + c_c - 2 g_j) (first round: assignment), then the chunk
// sums of d2; the last block draws r = draws[next] mod T and selects the
// chunk whose prefix range holds r.
__global__ __launch_bounds__(kBlock) void k_seed_update(int F, const double* __restrict__ colnorm,
                                                        const double* __restrict__ gram,
                                                        const int* __restrict__ finv,
                                                        const int* centres, int slot, int first,
                                                        long long* __restrict__ d2,
                                                        long long* __restrict__ chunk_sum,
                                                        const unsigned long long* draws, int next,
                                                        SeedState* st, unsigned* ticket) {
  if (st->stop) return;
  __shared__ long long red[kBlock];
  __shared__ int is_last;
  // d2 and the draw run over features in the caller's order; colnorm and
  // gram are held in the internal order
  const long long cc = (long long)colnorm[finv[centres[slot]]];
  long long sum = 0;
  const int j0 = blockIdx.x * kSeedChunk;
  for (int j = j0 + threadIdx.x; j < min(F, j0 + kSeedChunk); j += kBlock) {
    const int jn = finv[j];
    const long long dist = (long long)colnorm[jn] + cc - 2 * (long long)gram[jn];
    const long long v = first ? dist : min(d2[j], dist);
    d2[j] = v;
    sum += v;
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __hip_atomic_store(&chunk_sum[blockIdx.x], red[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wait_stores();
    const unsigned prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (next < 0) return;   // no further draw
  long long T = 0;
  for (int b = 0; b < (int)gridDim.x; ++b)
    T += __hip_atomic_load(&chunk_sum[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (T <= 0) {
    st->stop = 1;
    return;
  }
  const long long r = (long long)(draws[next] % (unsigned long long)T);
  long long acc = 0;
  int b = 0;
  for (; b < (int)gridDim.x; ++b) {
    const long long cs = __hip_atomic_load(&chunk_sum[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (acc + cs > r) break;
    acc += cs;
  }
  st->chunk = b;
  st->r_rem = r - acc;
}

// Smallest j in the selected chunk whose inclusive prefix of d2 exceeds r_rem.
__global__ __launch_bounds__(kSeedChunk) void k_seed_pick(int F, const long long* __restrict__ d2,
                                                          int* centres, int slot, SeedState* st) {
  if (st->stop) return;
  __shared__ long long sc[kSeedChunk];
  __shared__ int found;
  const int j = st->chunk * kSeedChunk + threadIdx.x;
  sc[threadIdx.x] = (j < F) ? d2[j] : 0;
  if (threadIdx.x == 0) found = INT_MAX;
  __syncthreads();
  for (int off = 1; off < kSeedChunk; off <<= 1) {
    const long long v = (threadIdx.x >= off) ? sc[threadIdx.x - off] : 0;
    __syncthreads();
    sc[threadIdx.x] += v;
    __syncthreads();
  }
  if (j < F && sc[threadIdx.x] > st->r_rem) atomicMin(&found, threadIdx.x);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (found == INT_MAX) {   // cannot happen when r_rem < the chunk sum
      st->stop = 1;
    } else {
      centres[slot] = st->chunk * kSeedChunk + found;
      st->n_centres = slot + 1;
    }
  }
}

// ----------------------------------------------------------------------------
// Lloyd
// ----------------------------------------------------------------------------
struct Item {
  int feature;
  int rb, re;   // rows [rb, re) of the feature's CSC column (offsets into row_idx)
  int heavy;    // index into the heavy histogram buffer, or -1
};

__global__ __launch_bounds__(kBlock) void k_count_members(int F, int k, const int* __restrict__ lab,
                                                          int* __restrict__ n) {
  extern __shared__ int hist[];
  for (int s = threadIdx.x; s < k; s += kBlock) hist[s] = 0;
  __syncthreads();
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const int l = lab[j];
    if (l >= 0) atomicAdd(&hist[l], 1);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < k; s += kBlock)
    if (hist[s]) atomicAdd(&n[s], hist[s]);
}

// Q_s = ||S_s||^2 = sum over rows of (count of cluster-s features in the row)^2.
__global__ __launch_bounds__(kBlock) void k_row_q(int N, int k, const int* __restrict__ row_ptr,
                                                  const int* __restrict__ col_idx,
                                                  const int* __restrict__ lab,
                                                  unsigned long long* __restrict__ Q,
                                                  int rows_per_block) {
  extern __shared__ unsigned long long qloc[];
  for (int s = threadIdx.x; s < k; s += kBlock) qloc[s] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r0 = blockIdx.x * rows_per_block;
  const int r1 = min(N, r0 + rows_per_block);
  for (int i = r0 + wid; i < r1; i += kBlock / 64) {
    const int a = row_ptr[i], b = row_ptr[i + 1];
    for (int a0 = a; a0 < b; a0 += 64) {
      const int ea = a0 + lane;
      const int La = (ea < b) ? lab[col_idx[ea]] : -1;
      int cnt = 0;
      bool first = true;
      for (int b0 = a; b0 < b; b0 += 64) {
        const int eb = b0 + lane;
        const int Lb = (eb < b) ? lab[col_idx[eb]] : -2;
        for (int t = 0; t < 64; ++t) {
          const int x = __shfl(Lb, t, 64);
          const bool eq = (x == La);
          cnt += eq ? 1 : 0;
          if (eq && (b0 + t) < ea) first = false;
        }
      }
      if (La >= 0 && first) atomicAdd(&qloc[La], (unsigned long long)cnt * (unsigned long long)cnt);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < k; s += kBlock)
    if (qloc[s]) atomicAdd(&Q[s], qloc[s]);
}

struct Cand {
  long long num;   // Q_s - 2 n_s h_s
  long long den;   // n_s^2 (> 0), or 0 for "none"
  int idx;
};

__device__ inline bool cand_less(const Cand& a, const Cand& b) {
  if (b.den == 0) return a.den != 0;
  if (a.den == 0) return false;
  const __int128 l = (__int128)a.num * b.den, r = (__int128)b.num * a.den;
  return l < r || (l == r && a.idx < b.idx);
}

__device__ inline Cand block_argmin(Cand c, Cand* lds) {
  lds[threadIdx.x] = c;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const Cand o = lds[threadIdx.x + off];
      if (cand_less(o, lds[threadIdx.x])) lds[threadIdx.x] = o;
    }
    __syncthreads();
  }
  const Cand r = lds[0];
  __syncthreads();
  return r;
}

// s0 = lowest index minimising Q_s / n_s^2 over non-empty clusters.
__global__ __launch_bounds__(kBlock) void k_s0(int k, const int* __restrict__ n,
                                               const unsigned long long* __restrict__ Q, int* s0) {
  __shared__ Cand lds[kBlock];
  Cand best{0, 0, INT_MAX};
  for (int s = threadIdx.x; s < k; s += kBlock) {
    if (n[s] > 0) {
      Cand c{(long long)Q[s], (long long)n[s] * n[s], s};
      if (cand_less(c, best)) best = c;
    }
  }
  best = block_argmin(best, lds);
  if (threadIdx.x == 0) *s0 = (best.idx < k) ? best.idx : 0;
}

enum { MODE_ASSIGN = 0, MODE_GRAM = 1 };

// One block per work item: histogram of the labels of the features sharing
// a row with feature j, over the item's rows; then (assign) the exact argmin
// for a whole feature, or the partial histogram of a heavy feature; or
// (gram) the row label_j of S^T S += histogram.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_two_hop(
    int k, const Item* __restrict__ items, const int* __restrict__ row_ptr,
    const int* __restrict__ col_idx, const int* __restrict__ row_idx,
    const int* __restrict__ lab, const int* __restrict__ n,
    const unsigned long long* __restrict__ Q, const int* s0p, int* __restrict__ lab_new,
    int* __restrict__ heavy_hist, unsigned long long* __restrict__ StS, int* changed) {
  extern __shared__ int smem[];
  int* hist = smem;          // [k]
  int* touched = smem + k;   // [k]
  __shared__ int ntouched;
  __shared__ Cand lds[kBlock];
  const Item it = items[blockIdx.x];
  for (int s = threadIdx.x; s < k; s += kBlock) hist[s] = 0;
  if (threadIdx.x == 0) ntouched = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int e = it.rb + wid; e < it.re; e += kBlock / 64) {
    const int i = row_idx[e];
    const int a = row_ptr[i], b = row_ptr[i + 1];
    for (int q = a + lane; q < b; q += 64) {
      const int l = lab[col_idx[q]];
      if (l >= 0) {
        if (atomicAdd(&hist[l], 1) == 0) touched[atomicAdd(&ntouched, 1)] = l;
      }
    }
  }
  __syncthreads();
  const int nt = ntouched;
  if (MODE == MODE_GRAM) {
    const int lj = lab[it.feature];
    for (int t = threadIdx.x; t < nt; t += kBlock) {
      const int s = touched[t];
      atomicAdd(&StS[(size_t)lj * k + s], (unsigned long long)hist[s]);
    }
    return;
  }
  if (it.heavy >= 0) {
    for (int t = threadIdx.x; t < nt; t += kBlock) {
      const int s = touched[t];
      atomicAdd(&heavy_hist[(size_t)it.heavy * k + s], hist[s]);
    }
    return;
  }
  Cand best{0, 0, INT_MAX};
  for (int t = threadIdx.x; t <= nt; t += kBlock) {
    const int s = (t < nt) ? touched[t] : *s0p;
    const long long ns = n[s];
    if (ns > 0) {
      Cand c{(long long)Q[s] - 2 * ns * (long long)hist[s], ns * ns, s};
      if (cand_less(c, best)) best = c;
    }
  }
  best = block_argmin(best, lds);
  if (threadIdx.x == 0) {
    lab_new[it.feature] = best.idx;
    if (best.idx != lab[it.feature]) atomicAdd(changed, 1);
  }
}

// Heavy features: argmin over all clusters from the summed chunk histograms.
__global__ __launch_bounds__(kBlock) void k_heavy_final(int k, const int* __restrict__ heavy_feat,
                                                        int* __restrict__ heavy_hist,
                                                        const int* __restrict__ lab,
                                                        const int* __restrict__ n,
                                                        const unsigned long long* __restrict__ Q,
                                                        int* __restrict__ lab_new, int* changed) {
  __shared__ Cand lds[kBlock];
  const int h = blockIdx.x;
  const int j = heavy_feat[h];
  int* hh = heavy_hist + (size_t)h * k;
  Cand best{0, 0, INT_MAX};
  for (int s = threadIdx.x; s < k; s += kBlock) {
    const long long ns = n[s];
    const long long hs = hh[s];
    hh[s] = 0;
    if (ns > 0) {
      Cand c{(long long)Q[s] - 2 * ns * hs, ns * ns, s};
      if (cand_less(c, best)) best = c;
    }
  }
  best = block_argmin(best, lds);
  if (threadIdx.x == 0) {
    lab_new[j] = best.idx;
    if (best.idx != lab[j]) atomicAdd(changed, 1);
  }
}

__global__ void k_init_labels(int F, int nc, const int* centres, int* lab) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) lab[j] = -1;
  // centres are written by a second launch (ordering across blocks)
}
__global__ void k_set_centres(int nc, const int* centres, const int* finv, int* lab) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nc) lab[finv[centres[s]]] = s;
}

// Compaction: remap[s] = rank of s among non-empty clusters.  One block.
__global__ __launch_bounds__(1024) void k_compact(int k, const int* n, int* remap, int* fc) {
  __shared__ int pre[1024];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int s0 = 0; s0 < k; s0 += 1024) {
    const int s = s0 + threadIdx.x;
    const int f = (s < k && n[s] > 0) ? 1 : 0;
    pre[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int v = (threadIdx.x >= off) ? pre[threadIdx.x - off] : 0;
      __syncthreads();
      pre[threadIdx.x] += v;
      __syncthreads();
    }
    if (s < k) remap[s] = f ? base + pre[threadIdx.x] - 1 : -1;
    __syncthreads();
    if (threadIdx.x == 1023) base += pre[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *fc = base;
}

__global__ void k_relabel(int F, const int* remap, int* lab, int* bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F) return;
  const int l = lab[j];
  const int m = (l >= 0) ? remap[l] : -1;
  if (m < 0) atomicOr(bad, 1);
  lab[j] = m;
}

__global__ void k_check_labels(int F, int nlab, const int* lab_in, const int* fperm, int* lab,
                               int* bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F) return;
  const int l = lab_in[fperm[j]];
  if (l < 0 || l >= nlab) atomicOr(bad, 1);
  lab[j] = l;
}

__global__ void k_scale(int fc, const int* n, double* scale) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < fc) scale[s] = 1.0 / sqrt((double)n[s]);
}

__global__ void k_gram_scale(int fc, const unsigned long long* StS, const double* scale, double* K) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)fc * fc) return;
  const int s = (int)(t / fc), u = (int)(t % fc);
  K[t] = (double)StS[t] * scale[s] * scale[u];
}

__global__ void k_iota_f(int* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

// off[s] = first position of key >= s in the sorted keys (s in [0, nseg]).
__global__ void k_offsets(const int* keys, int n, int nseg, int* off) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nseg) return;
  int lo = 0, hi = n;
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (keys[m] < s)
      lo = m + 1;
    else
      hi = m;
  }
  off[s] = lo;
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------
uint64_t splitmix64_next(uint64_t& state) {
  // SplitMix64 (Steele, Lea & Flood 2014)
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct KmWork {
  std::vector<Item> items;
  std::vector<int> heavy_feat;
  Item* d_items = nullptr;
  int* d_heavy_feat = nullptr;
  int* d_heavy_hist = nullptr;
  ~KmWork() {
    if (d_items) (void)dev_free(d_items);
    if (d_heavy_feat) (void)dev_free(d_heavy_feat);
    if (d_heavy_hist) (void)dev_free(d_heavy_hist);
  }
};

// Work items: whole columns, or chunks of at most `chunk_rows` rows for long
// columns (their histograms are summed in a global buffer).
static rr_status make_items(rr_handle* h, KmWork& kw, int k, bool need_heavy, hipStream_t s) {
  const Sparse& X = h->X;
  std::vector<int> cp(X.F + 1);
  RR_HIP(hipMemcpyAsync(cp.data(), X.col_ptr, sizeof(int) * (X.F + 1), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  const double avg_row = X.N ? (double)X.nnz / X.N : 1.0;
  const int chunk_rows = std::max(64, (int)(16384.0 / std::max(1.0, avg_row)));
  kw.items.clear();
  kw.heavy_feat.clear();
  for (int j = 0; j < X.F; ++j) {
    const int a = cp[j], b = cp[j + 1];
    if (b - a <= chunk_rows || !need_heavy) {
      kw.items.push_back(Item{j, a, b, -1});
    } else {
      const int hidx = (int)kw.heavy_feat.size();
      kw.heavy_feat.push_back(j);
      for (int r = a; r < b; r += chunk_rows) kw.items.push_back(Item{j, r, std::min(b, r + chunk_rows), hidx});
    }
  }
  RR_HIP(dmalloc(&kw.d_items, sizeof(Item) * std::max<size_t>(1, kw.items.size())));
  RR_HIP(hipMemcpyAsync(kw.d_items, kw.items.data(), sizeof(Item) * kw.items.size(),
                        hipMemcpyHostToDevice, s));
  if (!kw.heavy_feat.empty()) {
    RR_HIP(dmalloc(&kw.d_heavy_feat, sizeof(int) * kw.heavy_feat.size()));
    RR_HIP(hipMemcpyAsync(kw.d_heavy_feat, kw.heavy_feat.data(), sizeof(int) * kw.heavy_feat.size(),
                          hipMemcpyHostToDevice, s));
    RR_HIP(dmalloc(&kw.d_heavy_hist, sizeof(int) * kw.heavy_feat.size() * (size_t)k));
    RR_HIP(hipMemsetAsync(kw.d_heavy_hist, 0, sizeof(int) * kw.heavy_feat.size() * (size_t)k, s));
  }
  RR_HIP(hipStreamSynchronize(s));
  return RR_OK;
}

static size_t two_hop_lds(int k) { return sizeof(int) * 2 * (size_t)k; }

rr_status run_kmeans(rr_handle* h, int k, uint64_t seed, int max_iter, hipStream_t s) {
  const Sparse& X = h->X;
  const int F = X.F, N = X.N;
  if (!X.binary) return fail(RR_ERR_UNSUPPORTED, "k-means on the GPU needs a binary X; pass labels_in");
  k = std::min(k, F);
  RR_TRY(check_coarse_size(k));
  // ---- seeding ----
  std::vector<unsigned long long> draws(k);
  uint64_t st_rng = seed;
  for (int i = 0; i < k; ++i) draws[i] = splitmix64_next(st_rng);
  unsigned long long* d_draws = nullptr;
  long long *d2 = nullptr, *chunk_sum = nullptr;
  double *ind = nullptr, *gram = nullptr;
  SeedState* st = nullptr;
  unsigned* ticket = nullptr;
  const int nchunks = cdiv(F, kSeedChunk);
  RR_HIP(dmalloc(&d_draws, sizeof(unsigned long long) * k));
  RR_HIP(dmalloc(&d2, sizeof(long long) * F));
  RR_HIP(dmalloc(&chunk_sum, sizeof(long long) * nchunks));
  RR_HIP(dmalloc(&ind, sizeof(double) * N));
  RR_HIP(dmalloc(&gram, sizeof(double) * F));
  RR_HIP(dmalloc(&st, sizeof(SeedState)));
  RR_HIP(dmalloc(&ticket, sizeof(unsigned)));
  RR_HIP(hipMemsetAsync(ticket, 0, sizeof(unsigned), s));
  RR_HIP(hipMemsetAsync(st, 0, sizeof(SeedState), s));
  RR_HIP(hipMemcpyAsync(d_draws, draws.data(), sizeof(unsigned long long) * k, hipMemcpyHostToDevice, s));
  launch_fill(ind, 0.0, N, s);
  k_seed_first<<<1, 64, 0, s>>>(d_draws, F, h->centres, st);
  Epi e{};
  e.out = gram;
  const int ind_grid = 64;
  for (int i = 0; i < k; ++i) {
    if (i > 0)
      k_indicator<<<ind_grid, kBlock, 0, s>>>(X.col_ptr, X.row_idx, h->centres, h->finv, i - 1, 0.0, ind, st);
    k_indicator<<<ind_grid, kBlock, 0, s>>>(X.col_ptr, X.row_idx, h->centres, h->finv, i, 1.0, ind, st);
    launch_csc(X, ind, EPI_STORE, e, &st->stop, s);
    const int next = (i + 1 < k) ? i + 1 : -1;
    k_seed_update<<<nchunks, kBlock, 0, s>>>(F, h->colnorm, gram, h->finv, h->centres, i, i == 0, d2,
                                             chunk_sum, d_draws, next, st, ticket);
    if (next > 0) k_seed_pick<<<1, kSeedChunk, 0, s>>>(F, d2, h->centres, next, st);
  }
  SeedState hst{};
  RR_HIP(hipMemcpyAsync(&hst, st, sizeof(SeedState), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  const int nc = hst.n_centres;
  h->n_centres = nc;
  RR_HIP(dev_free(d_draws));
  RR_HIP(dev_free(d2));
  RR_HIP(dev_free(chunk_sum));
  RR_HIP(dev_free(ind));
  RR_HIP(dev_free(gram));
  RR_HIP(dev_free(st));
  RR_HIP(dev_free(ticket));

  // ---- Lloyd ----
  KmWork kw;
  RR_TRY(make_items(h, kw, nc, true, s));
  int *lab = h->labels, *lab_new = nullptr, *n = nullptr, *s0 = nullptr, *changed = nullptr;
  unsigned long long* Q = nullptr;
  RR_HIP(dmalloc(&lab_new, sizeof(int) * F));
  RR_HIP(dmalloc(&n, sizeof(int) * nc));
  RR_HIP(dmalloc(&Q, sizeof(unsigned long long) * nc));
  RR_HIP(dmalloc(&s0, sizeof(int)));
  RR_HIP(dmalloc(&changed, sizeof(int)));
  k_init_labels<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, nc, h->centres, lab);
  k_set_centres<<<cdiv(nc, kBlock), kBlock, 0, s>>>(nc, h->centres, h->finv, lab);
  const int rows_per_block = 64;
  const int cnt_grid = std::min(1024, cdiv(F, kBlock));
  int it = 0;
  while (it < max_iter) {
    RR_HIP(hipMemsetAsync(n, 0, sizeof(int) * nc, s));
    RR_HIP(hipMemsetAsync(Q, 0, sizeof(unsigned long long) * nc, s));
    RR_HIP(hipMemsetAsync(changed, 0, sizeof(int), s));
    k_count_members<<<cnt_grid, kBlock, sizeof(int) * nc, s>>>(F, nc, lab, n);
    k_row_q<<<cdiv(N, rows_per_block), kBlock, sizeof(unsigned long long) * nc, s>>>(
        N, nc, X.row_ptr, X.col_idx, lab, Q, rows_per_block);
    k_s0<<<1, kBlock, 0, s>>>(nc, n, Q, s0);
    k_two_hop<MODE_ASSIGN><<<(int)kw.items.size(), kBlock, two_hop_lds(nc), s>>>(
        nc, kw.d_items, X.row_ptr, X.col_idx, X.row_idx, lab, n, Q, s0, lab_new,
        kw.d_heavy_hist, nullptr, changed);
    if (!kw.heavy_feat.empty())
      k_heavy_final<<<(int)kw.heavy_feat.size(), kBlock, 0, s>>>(nc, kw.d_heavy_feat,
                                                                  kw.d_heavy_hist, lab, n, Q,
                                                                  lab_new, changed);
    int hchanged = 0;
    RR_HIP(hipMemcpyAsync(&hchanged, changed, sizeof(int), hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
    std::swap(lab, lab_new);
    ++it;
    if (hchanged == 0) break;
  }
  h->kmeans_iters = it;
  if (lab != h->labels) {
    RR_HIP(hipMemcpyAsync(h->labels, lab, sizeof(int) * F, hipMemcpyDeviceToDevice, s));
    std::swap(lab, lab_new);   // lab_new now points at the scratch buffer
  }
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(lab_new));
  RR_HIP(dev_free(n));
  RR_HIP(dev_free(Q));
  RR_HIP(dev_free(s0));
  RR_HIP(dev_free(changed));
  return set_labels(h, nullptr, nc, s);
}

// Finalise an aggregation held in h->labels (or copied from labels_in):
// drop empty clusters, renumber, sizes, scales, the cluster-sorted
// permutation and its restriction plan.
__global__ void k_inverse_perm(const int* __restrict__ perm, int F, int* __restrict__ inv) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < F) inv[perm[k]] = k;
}

rr_status set_labels(rr_handle* h, const int* labels_in, int nlab, hipStream_t s) {
  const int F = h->X.F;
  int* bad = nullptr;
  int *n = nullptr, *remap = nullptr, *fc = nullptr;
  RR_HIP(dmalloc(&bad, sizeof(int)));
  RR_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  if (labels_in)
    k_check_labels<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, nlab, labels_in, h->fperm, h->labels, bad);
  RR_HIP(dmalloc(&n, sizeof(int) * nlab));
  RR_HIP(dmalloc(&remap, sizeof(int) * nlab));
  RR_HIP(dmalloc(&fc, sizeof(int)));
  RR_HIP(hipMemsetAsync(n, 0, sizeof(int) * nlab, s));
  int hbad = 0;
  RR_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  if (hbad) return fail(RR_ERR_INVALID_ARG, "labels_in: label outside [0, n_labels_in)");
  if ((size_t)nlab * 4 > 150 * 1024) return fail(RR_ERR_UNSUPPORTED, "too many labels");
  k_count_members<<<std::min(1024, cdiv(F, kBlock)), kBlock, sizeof(int) * nlab, s>>>(F, nlab, h->labels, n);
  k_compact<<<1, 1024, 0, s>>>(nlab, n, remap, fc);
  k_relabel<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, remap, h->labels, bad);
  int hfc = 0;
  RR_HIP(hipMemcpyAsync(&hfc, fc, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(n));
  RR_HIP(dev_free(remap));
  RR_HIP(dev_free(fc));
  RR_HIP(dev_free(bad));
  if (hbad) return fail(RR_ERR_DEVICE, "internal: unassigned feature after clustering");
  h->FC = hfc;
  RR_HIP(dmalloc(&h->csize, sizeof(int) * hfc));
  RR_HIP(dmalloc(&h->cscale, sizeof(double) * hfc));
  RR_HIP(dmalloc(&h->perm, sizeof(int) * F));
  RR_HIP(dmalloc(&h->coff, sizeof(int) * (hfc + 1)));
  RR_HIP(hipMemsetAsync(h->csize, 0, sizeof(int) * hfc, s));
  k_count_members<<<std::min(1024, cdiv(F, kBlock)), kBlock, sizeof(int) * hfc, s>>>(F, hfc, h->labels, h->csize);
  k_scale<<<cdiv(hfc, kBlock), kBlock, 0, s>>>(hfc, h->csize, h->cscale);
  // perm: features sorted by cluster, stable
  int *keys_out = nullptr, *iota = nullptr;
  RR_HIP(dmalloc(&keys_out, sizeof(int) * F));
  RR_HIP(dmalloc(&iota, sizeof(int) * F));
  k_iota_f<<<cdiv(F, kBlock), kBlock, 0, s>>>(iota, F);
  size_t tmp_bytes = 0;
  unsigned end_bit = 1;
  while ((1ll << end_bit) < (long long)hfc) ++end_bit;
  RR_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, h->labels, keys_out, iota, h->perm, (size_t)F, 0u, end_bit, s));
  void* tmp = nullptr;
  RR_HIP(dmalloc(&tmp, std::max<size_t>(tmp_bytes, 1)));
  RR_HIP(rocprim::radix_sort_pairs(tmp, tmp_bytes, h->labels, keys_out, iota, h->perm, (size_t)F, 0u, end_bit, s));
  k_offsets<<<cdiv(hfc + 1, kBlock), kBlock, 0, s>>>(keys_out, F, hfc, h->coff);
  // cpos: the inverse of perm (where each feature sits in cluster order)
  RR_HIP(dmalloc(&h->cpos, sizeof(int) * F));
  k_inverse_perm<<<cdiv(F, kBlock), kBlock, 0, s>>>(h->perm, F, h->cpos);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(tmp));
  RR_HIP(dev_free(keys_out));
  RR_HIP(dev_free(iota));
  RR_TRY(build_merge_plan(h->restrict_plan, h->coff + 1, h->coff, hfc, F, s));
  return build_chunk_plan(h->restrict_plan, h->coff, hfc, s);
}

// K = diag(n)^-1/2 S^T S diag(n)^-1/2 with S = X P_u (binary X: exact
// integer S^T S accumulated from per-feature label histograms).
rr_status build_coarse_gram(rr_handle* h, hipStream_t s) {
  const Sparse& X = h->X;
  const int fc = h->FC;
  if (!X.binary) return build_coarse_gram_valued(h, s);
  RR_TRY(check_coarse_size(fc));   // before anything is allocated
  KmWork kw;
  RR_TRY(make_items(h, kw, fc, false, s));
  unsigned long long* StS = nullptr;
  const size_t nn = (size_t)fc * fc;
  RR_HIP(dmalloc(&StS, sizeof(unsigned long long) * nn));
  hipError_t e = hipMemsetAsync(StS, 0, sizeof(unsigned long long) * nn, s);
  if (e == hipSuccess) {
    k_two_hop<MODE_GRAM><<<(int)kw.items.size(), kBlock, two_hop_lds(fc), s>>>(
        fc, kw.d_items, X.row_ptr, X.col_idx, X.row_idx, h->labels, nullptr, nullptr, nullptr,
        nullptr, nullptr, StS, nullptr);
    k_gram_scale<<<cdiv((long long)nn, kBlock), kBlock, 0, s>>>(fc, StS, h->cscale, h->K);
    e = hipStreamSynchronize(s);
  }
  (void)dev_free(StS);
  RR_HIP(e);
  return RR_OK;
}

// The exact integer Gram of 0/1 X keeps one histogram bin per cluster in
// LDS (8 bytes each beside the block's reduction space): at most 18,944
// clusters.
rr_status check_coarse_size(int fc) {
  if (two_hop_lds(fc) + 8 * kBlock > 150 * 1024)
    return fail(RR_ERR_UNSUPPORTED, "more than 18,944 clusters: too many for the LDS histogram of "
                                    "the coarse Gram matrix");
  return RR_OK;
}

}  // namespace rr
