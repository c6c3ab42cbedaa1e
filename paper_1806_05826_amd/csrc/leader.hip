// Leader-follower clustering of the feature columns (the leader-follower
// subsection of the paper's clustering section; the form of its
// experiments: Euclidean distance, leaders not updated), for 0/1 X in exact
// integer arithmetic.  The features are visited in the caller's order; each
// follows its nearest earlier leader (ties: the earliest) if that lies
// strictly within the tolerance, else it becomes the next leader.
//
// The scan runs over windows of kLfWin features.  For every feature of a
// window, one workgroup finds its nearest leader among those created before
// the window: co-occurrence counts with the leaders in its rows (per-row
// leader tables, a histogram in the workgroup's scratch), d^2 = c_f + c_s -
// 2 |f n s|, and the leader of smallest norm as the candidate for leaders
// sharing no row with it.  One workgroup then walks the window in order,
// taking every follower decision, and stops at the first new leader: that
// leader enters the row tables of its rows, its co-occurrence with the rest
// of the window is counted, and those features' candidates are updated
// before the walk resumes.  A candidate is packed as (d^2 << 31) | leader,
// so the smaller key is the nearer leader, the earlier one on ties.
#include <algorithm>
#include <vector>

#include "rr_device.h"

namespace rr {

namespace {

constexpr int kLfWin = 256;
constexpr int kLfThreads = 256;
constexpr unsigned long long kNoLeader = ~0ull;
constexpr unsigned long long kLeaderMask = (1ull << 31) - 1;

struct LfState {
  int n_lead;       // leaders so far
  int minnorm;      // smallest leader norm and that leader (the earliest)
  int minnorm_id;
  int stop;         // walk: window position of the new leader, or the window size
  int new_f;        // that feature (internal index)
};

__device__ inline unsigned long long lf_key(long long d2, int s) {
  return ((unsigned long long)d2 << 31) | (unsigned long long)s;
}

__global__ void k_fill_int(int* x, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_lf_setpos(int t0, int nwin, const int* __restrict__ finv, int* winpos, int val_is_pos) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nwin) winpos[finv[t0 + q]] = val_is_pos ? q : -1;
}

__global__ __launch_bounds__(kLfThreads) void k_lf_best(int t0, const int* __restrict__ finv,
                                                        const int* __restrict__ col_ptr,
                                                        const int* __restrict__ row_idx,
                                                        const int* __restrict__ row_ptr,
                                                        const int* __restrict__ rl_cnt,
                                                        const int* __restrict__ rl_ids,
                                                        const int* __restrict__ lead_norm,
                                                        const LfState* __restrict__ st, int F, int* hist,
                                                        int* touched, unsigned long long* best) {
  const int w = blockIdx.x;
  const int f = finv[t0 + w];
  int* H = hist + (size_t)w * F;
  int* T = touched + (size_t)w * F;
  __shared__ int ntouch;
  __shared__ unsigned long long red[kLfThreads / 64];
  if (threadIdx.x == 0) ntouch = 0;
  __syncthreads();
  const int a = col_ptr[f], z = col_ptr[f + 1];
  for (int p = a + threadIdx.x; p < z; p += kLfThreads) {
    const int i = row_idx[p];
    const int r0 = row_ptr[i], c = rl_cnt[i];
    for (int k = 0; k < c; ++k) {
      const int s = rl_ids[r0 + k];
      if (atomicAdd(&H[s], 1) == 0) T[atomicAdd(&ntouch, 1)] = s;
    }
  }
  __syncthreads();
  const int nt = ntouch;
  const long long nf = z - a;
  unsigned long long bk = kNoLeader;
  for (int q = threadIdx.x; q < nt; q += kLfThreads) {
    const int s = T[q];
    const int c = __hip_atomic_load(&H[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&H[s], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bk = min(bk, lf_key(nf + lead_norm[s] - 2LL * c, s));
  }
  if (threadIdx.x == 0 && st->n_lead > 0) bk = min(bk, lf_key(nf + st->minnorm, st->minnorm_id));
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(bk, off, 64);
    bk = min(bk, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = bk;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
    for (int k = 1; k < kLfThreads / 64; ++k) m = min(m, red[k]);
    best[w] = m;
  }
}

// The window's decisions in order from position p0, up to the first new
// leader (one workgroup: the window's candidates and norms are staged in LDS,
// then one thread walks).
__global__ __launch_bounds__(kLfThreads) void k_lf_walk(int t0, int p0, int nwin, const int* __restrict__ finv,
                                                        const int* __restrict__ col_ptr, double tol2,
                                                        const unsigned long long* __restrict__ best,
                                                        LfState* st, int* labels, int* lead_norm,
                                                        int* lead_caller) {
  __shared__ unsigned long long bk[kLfWin];
  __shared__ int fi[kLfWin], nf[kLfWin];
  for (int q = threadIdx.x; q < nwin; q += kLfThreads) {
    bk[q] = best[q];
    const int f = finv[t0 + q];
    fi[q] = f;
    nf[q] = col_ptr[f + 1] - col_ptr[f];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int p = p0; p < nwin; ++p) {
    const unsigned long long k = bk[p];
    if (k != kNoLeader && (double)(long long)(k >> 31) < tol2) {
      labels[fi[p]] = (int)(k & kLeaderMask);
      continue;
    }
    const int s = st->n_lead;
    st->n_lead = s + 1;
    labels[fi[p]] = s;
    lead_norm[s] = nf[p];
    lead_caller[s] = t0 + p;
    if (s == 0 || nf[p] < st->minnorm) {
      st->minnorm = nf[p];
      st->minnorm_id = s;
    }
    st->stop = p;
    st->new_f = fi[p];
    return;
  }
  st->stop = nwin;
}

// The new leader s (feature g) enters the leader tables of its rows; its
// co-occurrence with the window's features after position p is counted.
__global__ __launch_bounds__(kLfThreads) void k_lf_add_leader(int g, int s, int p, const int* __restrict__ col_ptr,
                                                              const int* __restrict__ row_idx,
                                                              const int* __restrict__ row_ptr,
                                                              const int* __restrict__ col_idx, int* rl_cnt,
                                                              int* rl_ids, const int* __restrict__ winpos,
                                                              int* wcnt) {
  const int a = col_ptr[g], z = col_ptr[g + 1];
  for (int e = a + blockIdx.x * kLfThreads + threadIdx.x; e < z; e += gridDim.x * kLfThreads) {
    const int i = row_idx[e];
    const int r0 = row_ptr[i], r1 = row_ptr[i + 1];
    const int k = atomicAdd(&rl_cnt[i], 1);
    rl_ids[r0 + k] = s;
    for (int c = r0; c < r1; ++c) {
      const int q = winpos[col_idx[c]];
      if (q > p) atomicAdd(&wcnt[q], 1);
    }
  }
}

// The window's candidates after position p against the new leader s.
__global__ __launch_bounds__(kLfThreads) void k_lf_merge(int s, int t0, int p, int nwin, const int* __restrict__ finv,
                                                         const int* __restrict__ col_ptr,
                                                         const int* __restrict__ lead_norm, int* wcnt,
                                                         unsigned long long* best) {
  for (int q = p + 1 + threadIdx.x; q < nwin; q += kLfThreads) {
    const int f = finv[t0 + q];
    const int c = __hip_atomic_load(&wcnt[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wcnt[q] = 0;
    const long long nfv = col_ptr[f + 1] - col_ptr[f];
    const unsigned long long k = lf_key(nfv + lead_norm[s] - 2LL * c, s);
    if (k < best[q]) best[q] = k;
  }
}

}  // namespace

// Labels (internal order, in h->labels) and leaders (caller indices, in
// h->centres) of the leader-follower scan at tolerance tol; *fc receives the
// number of clusters.  Setup only.
rr_status leader_follower(rr_handle* h, double tol, int* fc, hipStream_t s) {
  const Sparse& X = h->X;
  if (!X.binary) return fail(RR_ERR_UNSUPPORTED, "leader-follower clustering is built for 0/1 X");
  const int F = X.F, N = X.N;
  const double tol2 = tol * tol;
  int *rl_cnt = nullptr, *rl_ids = nullptr, *lead_norm = nullptr, *winpos = nullptr, *wcnt = nullptr;
  int *hist = nullptr, *touched = nullptr;
  unsigned long long* best = nullptr;
  LfState* st = nullptr;
  RR_HIP(dmalloc(&rl_cnt, sizeof(int) * std::max(1, N)));
  RR_HIP(dmalloc(&rl_ids, sizeof(int) * std::max(1, X.nnz)));
  RR_HIP(dmalloc(&lead_norm, sizeof(int) * F));
  RR_HIP(dmalloc(&winpos, sizeof(int) * F));
  RR_HIP(dmalloc(&wcnt, sizeof(int) * kLfWin));
  RR_HIP(dmalloc(&hist, sizeof(int) * (size_t)kLfWin * F));
  RR_HIP(dmalloc(&touched, sizeof(int) * (size_t)kLfWin * F));
  RR_HIP(dmalloc(&best, sizeof(unsigned long long) * kLfWin));
  RR_HIP(dmalloc(&st, sizeof(LfState)));
  if (!h->centres) RR_HIP(dmalloc(&h->centres, sizeof(int) * F));
  RR_HIP(hipMemsetAsync(rl_cnt, 0, sizeof(int) * std::max(1, N), s));
  RR_HIP(hipMemsetAsync(wcnt, 0, sizeof(int) * kLfWin, s));
  RR_HIP(hipMemsetAsync(hist, 0, sizeof(int) * (size_t)kLfWin * F, s));
  RR_HIP(hipMemsetAsync(st, 0, sizeof(LfState), s));
  k_fill_int<<<cdiv(F, kLfThreads), kLfThreads, 0, s>>>(winpos, -1, F);
  LfState hs{};
  rr_status status = RR_OK;
  for (int t0 = 0; t0 < F && status == RR_OK; t0 += kLfWin) {
    const int nwin = std::min(kLfWin, F - t0);
    k_lf_setpos<<<cdiv(nwin, kLfThreads), kLfThreads, 0, s>>>(t0, nwin, h->finv, winpos, 1);
    k_lf_best<<<nwin, kLfThreads, 0, s>>>(t0, h->finv, X.col_ptr, X.row_idx, X.row_ptr, rl_cnt, rl_ids,
                                          lead_norm, st, F, hist, touched, best);
    int p0 = 0;
    for (;;) {
      k_lf_walk<<<1, kLfThreads, 0, s>>>(t0, p0, nwin, h->finv, X.col_ptr, tol2, best, st, h->labels, lead_norm,
                                         h->centres);
      if (hipMemcpyAsync(&hs, st, sizeof(LfState), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        status = fail(RR_ERR_DEVICE, "leader-follower: reading the scan state");
        break;
      }
      if (hs.stop >= nwin) break;
      const int g = hs.new_f, sl = hs.n_lead - 1, p = hs.stop;
      if (g < 0 || g >= F || p < p0 || p >= nwin) {
        status = fail(RR_ERR_DEVICE, "internal: leader-follower state out of range");
        break;
      }
      int ng = 0;
      RR_HIP(hipMemcpyAsync(&ng, X.col_ptr + g, sizeof(int), hipMemcpyDeviceToHost, s));
      int ng1 = 0;
      RR_HIP(hipMemcpyAsync(&ng1, X.col_ptr + g + 1, sizeof(int), hipMemcpyDeviceToHost, s));
      RR_HIP(hipStreamSynchronize(s));
      const int grid = std::max(1, std::min(1024, cdiv(ng1 - ng, kLfThreads)));
      k_lf_add_leader<<<grid, kLfThreads, 0, s>>>(g, sl, p, X.col_ptr, X.row_idx, X.row_ptr, X.col_idx, rl_cnt,
                                                  rl_ids, winpos, wcnt);
      k_lf_merge<<<1, kLfThreads, 0, s>>>(sl, t0, p, nwin, h->finv, X.col_ptr, lead_norm, wcnt, best);
      p0 = p + 1;
    }
    k_lf_setpos<<<cdiv(nwin, kLfThreads), kLfThreads, 0, s>>>(t0, nwin, h->finv, winpos, 0);
  }
  (void)hipStreamSynchronize(s);
  (void)dev_free(rl_cnt); (void)dev_free(rl_ids); (void)dev_free(lead_norm); (void)dev_free(winpos);
  (void)dev_free(wcnt); (void)dev_free(hist); (void)dev_free(touched); (void)dev_free(best); (void)dev_free(st);
  RR_TRY(status);
  RR_HIP(hipGetLastError());
  *fc = hs.n_lead;
  return RR_OK;
}

}  // namespace rr
