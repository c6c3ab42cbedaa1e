// Many independent ridge problems (0/1 X, FP64) solved in one persistent
// launch: every workgroup takes the next problem from a device queue (the
// problems sorted by descending cost, so the longest start first), runs its
// whole PCG solve with the two-level V(1,1) preconditioner (or Jacobi)
// using workgroup barriers only, writes w and the problem's record, and
// takes the next problem until the queue is empty.
//
// The operator q = X^T (X v) + lambda v of a problem runs out of LDS: the
// gathered vector v (F <= 8192 features, 64 KB of FP64) sits in LDS, and the
// rows are processed in chunks of kBU = 10240: the chunk's u = X v is formed
// in LDS (80 KB), then every column adds the entries of its rows inside the
// chunk (a column's CSC entries of chunk h start at csplit[h F + j]) into
// t_j.  A group of lanes owns a row (G_row lanes, the problem's tuned value)
// or a column (64, 16, 4 or 1 lanes by the column's length; the columns are
// in descending-count order, so each class is a range), adds in a fixed
// order and reduces with a fixed butterfly; the same group owns the same
// column in every chunk, so t_j accumulates without atomics and every result
// is bitwise reproducible.  Between operator applications the coarse
// residual and correction live in the chunk buffer.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>

#include "rr_device.h"

namespace rr {

constexpr int kBT = 1024;   // threads per workgroup
static_assert(kBT == kSliceBlock, "the batched solver runs 1024-thread workgroups");

// LDS: the gathered vector and the row chunk (or, between applications, the
// coarse residual and correction)
struct BatchLds {
  double V[kBatchFMax];
  double U[kBatchRows];
  double red[kBT / 64];
  int qslot;
};

__device__ inline double wg_sum(double v, double* red) { return block_sum_n<kBT>(v, red); }

// sum over groups of G lanes (G a power of two <= 64), fixed butterfly
template <int G>
__device__ inline double group_sum(double s) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
  return s;
}

// sum of vec[idx[k]] over k in [a, z) by the G lanes of a group, lane sub
// taking its share in a fixed order: the 4-aligned body [a4, z4) in groups
// of four entries (one 8-byte load each; group q goes to lane q mod G, 16
// loads, 64 entries, in flight per lane: one workgroup per CU streams the
// problem's indexes, so the bytes it keeps in flight bound it), then the
// unaligned head [a, a4) and tail [z4, z), one entry per lane; two
// accumulators.  idx is 8-byte aligned.
template <int G>
__device__ inline double lane_gather(const uint16_t* __restrict__ idx, const double* vec, int a, int z,
                                     int sub) {
  constexpr int B = 16;
  double s0 = 0.0, s1 = 0.0;
  const int a4 = min(z, (a + 3) & ~3);
  const int z4 = max(a4, z & ~3);
  const uint2* p = reinterpret_cast<const uint2*>(idx);
  const int qz = z4 >> 2;
  int q = (a4 >> 2) + sub;
  auto add4 = [&](uint2 w) {
    s0 += vec[w.x & 0xffffu];
    s1 += vec[w.x >> 16];
    s0 += vec[w.y & 0xffffu];
    s1 += vec[w.y >> 16];
  };
  for (; q + (B - 1) * G < qz; q += B * G) {
    uint2 w[B];
#pragma unroll
    for (int u = 0; u < B; ++u) w[u] = p[q + u * G];
#pragma unroll
    for (int u = 0; u < B; ++u) add4(w[u]);
  }
  if (q < qz) {   // the rest: fewer than 16 groups, loads issued together
    uint2 w[B];
#pragma unroll
    for (int u = 0; u < B; ++u) w[u] = (q + u * G < qz) ? p[q + u * G] : make_uint2(0xffffffffu, 0xffffffffu);
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (w[u].x != 0xffffffffu) add4(w[u]);
  }
  for (int k = a + sub; k < a4; k += G) s0 += vec[idx[k]];
  for (int k = z4 + sub; k < z; k += G) s1 += vec[idx[k]];
  return s0 + s1;
}

// rows [r0, r1) of the chunk: U[i - r0] = sum_{j in row i} V[j], G lanes per row
template <int G>
__device__ inline void chunk_rows(const BatchProb& P, BatchLds& L, int r0, int r1) {
  const int tid = threadIdx.x, sub = tid & (G - 1);
  constexpr int per = kBT / G;
  const int n = r1 - r0;
  for (int base = 0; base < n; base += per) {   // the same trip count in every lane
    const int i = r0 + base + tid / G;
    double s = 0.0;
    if (i < r1) s = lane_gather<G>(P.ci, L.V, P.rp[i], P.rp[i + 1], sub);
    s = group_sum<G>(s);
    if (i < r1 && sub == 0) L.U[i - r0] = s;
  }
}

// columns [c0, c1) over chunk h: t_j (+)= sum of U over the column's rows in
// the chunk, G lanes per column
template <int G>
__device__ inline void chunk_cols(const BatchProb& P, const BatchLds& L, int h, int r0, int c0, int c1,
                                  double* __restrict__ t) {
  const int tid = threadIdx.x, sub = tid & (G - 1);
  constexpr int per = kBT / G;
  const int F = P.F;
  for (int base = c0; base < c1; base += per) {
    const int j = base + tid / G;
    double s = 0.0;
    if (j < c1)
      s = lane_gather<G>(P.ri, L.U, P.csplit[(size_t)h * F + j], P.csplit[(size_t)(h + 1) * F + j], sub);
    s = group_sum<G>(s);
    if (j < c1 && sub == 0) t[j] = (h == 0 ? 0.0 : t[j]) + s;
  }
}

template <int G>
__device__ inline void all_cols(const BatchProb& P, const BatchLds& L, int h, int r0, double* t) {
  (void)G;
  chunk_cols<64>(P, L, h, r0, 0, P.cls[0], t);
  chunk_cols<16>(P, L, h, r0, P.cls[0], P.cls[1], t);
  chunk_cols<4>(P, L, h, r0, P.cls[1], P.cls[2], t);
  chunk_cols<1>(P, L, h, r0, P.cls[2], P.F, t);
}

// t = X^T (X V) with V already in LDS (and visible: the caller synchronised)
__device__ inline void wg_gram(const BatchProb& P, BatchLds& L, double* __restrict__ t) {
  for (int h = 0; h < P.nchunk; ++h) {
    const int r0 = h * kBatchRows, r1 = min(P.N, r0 + kBatchRows);
    switch (P.grow) {
      case 1: chunk_rows<1>(P, L, r0, r1); break;
      case 2: chunk_rows<2>(P, L, r0, r1); break;
      case 4: chunk_rows<4>(P, L, r0, r1); break;
      case 8: chunk_rows<8>(P, L, r0, r1); break;
      case 16: chunk_rows<16>(P, L, r0, r1); break;
      case 32: chunk_rows<32>(P, L, r0, r1); break;
      default: chunk_rows<64>(P, L, r0, r1); break;
    }
    __syncthreads();
    all_cols<1>(P, L, h, r0, t);
    __syncthreads();
  }
}

// t = X^T y for a caller vector y (rows of the chunk staged through U)
__device__ inline void wg_rhs(const BatchProb& P, BatchLds& L, const double* __restrict__ y,
                              double* __restrict__ t) {
  for (int h = 0; h < P.nchunk; ++h) {
    const int r0 = h * kBatchRows, r1 = min(P.N, r0 + kBatchRows);
    for (int i = r0 + threadIdx.x; i < r1; i += kBT) L.U[i - r0] = y[i];
    __syncthreads();
    all_cols<1>(P, L, h, r0, t);
    __syncthreads();
  }
}

// z = B r: V(1,1) two-level cycle (kind 1) or Jacobi (kind 0); returns <r,z>
__device__ inline double wg_precond(const BatchProb& P, BatchLds& L) {
  const int F = P.F, tid = threadIdx.x;
  const double lam = P.lam, om = P.omega;
  if (P.kind == 0) {
    double rz = 0.0;
    for (int j = tid; j < F; j += kBT) {
      const double zj = P.r[j] / (P.colnorm[j] + lam);
      P.z[j] = zj;
      rz += P.r[j] * zj;
    }
    return wg_sum(rz, L.red);
  }
  // e1 = w D^-1 r, into LDS and e1
  for (int j = tid; j < F; j += kBT) {
    const double e = (om * P.r[j]) / (P.colnorm[j] + lam);
    L.V[j] = e;
    P.e1[j] = e;
  }
  __syncthreads();
  wg_gram(P, L, P.t);
  // rho1 = r - (t + lam e1); c = P^T rho1 (cluster sums scaled by 1/sqrt(n_s)),
  // 16 lanes per cluster, into U[0, FC)
  {
    const int sub = tid & 15;
    for (int base = 0; base < P.FC; base += kBT / 16) {
      const int l = base + tid / 16;
      double s = 0.0;
      if (l < P.FC) {
        for (int k = P.coff[l] + sub; k < P.coff[l + 1]; k += 16) {
          const int j = P.perm[k];
          s += P.r[j] - (P.t[j] + lam * P.e1[j]);
        }
      }
      s = group_sum<16>(s);
      if (l < P.FC && sub == 0) L.U[l] = s * P.cscale[l];
    }
  }
  __syncthreads();
  // yc = A_c^-1 c, one wave per row, into U[FC, 2 FC)
  {
    const int wv = tid >> 6, lane = tid & 63;
    const int fc = P.FC;
    for (int row = wv; row < fc; row += kBT / 64) {
      const double* a = P.Ainv + (size_t)row * fc;
      double s0 = 0.0, s1 = 0.0;
      int c = lane;
      for (; c + 64 < fc; c += 128) {
        s0 += a[c] * L.U[c];
        s1 += a[c + 64] * L.U[c + 64];
      }
      if (c < fc) s0 += a[c] * L.U[c];
      double s = s0 + s1;
      s = group_sum<64>(s);
      if (lane == 0) L.U[fc + row] = s;
    }
  }
  __syncthreads();
  // e2 = e1 + P yc, into LDS and z
  for (int j = tid; j < F; j += kBT) {
    const int l = P.labels[j];
    const double e2 = P.e1[j] + P.cscale[l] * L.U[P.FC + l];
    L.V[j] = e2;
    P.z[j] = e2;
  }
  __syncthreads();
  wg_gram(P, L, P.t);
  // z = e2 + w D^-1 (r - (t + lam e2))
  double rz = 0.0;
  for (int j = tid; j < F; j += kBT) {
    const double e2 = L.V[j], rj = P.r[j];
    const double rho = rj - (P.t[j] + lam * e2);
    const double zj = e2 + (om * rho) / (P.colnorm[j] + lam);
    P.z[j] = zj;
    rz += rj * zj;
  }
  return wg_sum(rz, L.red);
}

__device__ inline void solve_one(const BatchProb& P, BatchLds& L, BatchOut* out) {
  const int F = P.F, tid = threadIdx.x;
  const double lam = P.lam;
  const long long t_begin = wall_clock64();
  // b
  if (P.rhs_is_b) {
    for (int j = tid; j < F; j += kBT) P.b[j] = P.rhs[P.fperm[j]];
  } else {
    wg_rhs(P, L, P.rhs, P.b);
  }
  __syncthreads();
  double bb = 0.0;
  for (int j = tid; j < F; j += kBT) {
    const double bj = P.b[j];
    P.x[j] = 0.0;
    P.r[j] = bj;
    bb += bj * bj;
  }
  bb = wg_sum(bb, L.red);
  int status = RR_ERR_NOT_CONVERGED, it = 0;
  double rr = bb, rz_keep = 0.0;
  if (bb == 0.0) {
    status = RR_OK;
  } else {
    double rz = wg_precond(P, L);
    for (int j = tid; j < F; j += kBT) P.p[j] = P.z[j];
    __syncthreads();
    if (!finite_pos(rz)) status = RR_ERR_BREAKDOWN;
    while (status == RR_ERR_NOT_CONVERGED && it < P.max_iter) {
      if (P.cap > 0 && it >= P.cap) {   // the host continues from x, r, p and rz
        status = kStatusYield;
        rz_keep = rz;
        break;
      }
      // q = A p (t holds X^T X p), <p, q>
      for (int j = tid; j < F; j += kBT) L.V[j] = P.p[j];
      __syncthreads();
      wg_gram(P, L, P.t);
      double pq = 0.0;
      for (int j = tid; j < F; j += kBT) pq += L.V[j] * (P.t[j] + lam * L.V[j]);
      pq = wg_sum(pq, L.red);
      if (!finite_pos(pq)) {
        status = RR_ERR_BREAKDOWN;
        break;
      }
      const double alpha = rz / pq;
      double rn = 0.0;
      for (int j = tid; j < F; j += kBT) {
        const double pj = L.V[j];
        P.x[j] += alpha * pj;
        const double rj = P.r[j] - alpha * (P.t[j] + lam * pj);
        P.r[j] = rj;
        rn += rj * rj;
      }
      rr = wg_sum(rn, L.red);
      ++it;
      if (!(rr == rr)) {
        status = RR_ERR_BREAKDOWN;
        break;
      }
      if (rr <= P.tol2 * bb) {
        status = RR_OK;
        break;
      }
      const double rz_new = wg_precond(P, L);
      if (!finite_pos(rz_new)) {
        status = RR_ERR_BREAKDOWN;
        break;
      }
      const double beta = rz_new / rz;
      rz = rz_new;
      for (int j = tid; j < F; j += kBT) P.p[j] = P.z[j] + beta * P.p[j];
      __syncthreads();
    }
  }
  if (status == kStatusYield) {
    if (tid == 0) {
      out->status = status;
      out->iters = it;
      out->relres = sqrt(rr / bb);
      out->true_relres = 0.0;
      out->rz = rz_keep;
      out->bb = bb;
      out->t_begin = t_begin;
      out->t_end = wall_clock64();
    }
    __syncthreads();
    return;
  }
  // w in the caller's order; the true residual ||b - A x||
  __syncthreads();
  for (int j = tid; j < F; j += kBT) L.V[j] = P.x[j];
  __syncthreads();
  for (int j = tid; j < F; j += kBT) P.w[j] = P.x[P.finv[j]];
  wg_gram(P, L, P.t);
  double tr = 0.0;
  for (int j = tid; j < F; j += kBT) {
    const double res = P.b[j] - (P.t[j] + lam * L.V[j]);
    tr += res * res;
  }
  tr = wg_sum(tr, L.red);
  if (tid == 0) {
    out->status = status;
    out->iters = it;
    out->relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    out->true_relres = bb > 0.0 ? sqrt(tr / bb) : 0.0;
    out->t_begin = t_begin;
    out->t_end = wall_clock64();
  }
  __syncthreads();
}

// Problems are taken in the order of `order` through the counter `queue`
// (zeroed by the launch sequence); every workgroup leaves once the counter
// has passed nprob, so the grid drains by itself.
__global__ __launch_bounds__(kBT) void k_batch_solve(const BatchProb* __restrict__ probs,
                                                     const int* __restrict__ order, int nprob,
                                                     int* queue, BatchOut* __restrict__ out) {
  __shared__ BatchLds L;
  for (;;) {
    if (threadIdx.x == 0) L.qslot = atomicAdd(queue, 1);
    __syncthreads();
    const int q = L.qslot;
    __syncthreads();
    if (q >= nprob) return;
    const int pi = order[q];
    solve_one(probs[pi], L, out + pi);
  }
}

// one operator application per problem (autotuning and timing): t = X^T X v
__global__ __launch_bounds__(kBT) void k_batch_gram(const BatchProb* __restrict__ probs, int nprob,
                                                    const double* const* __restrict__ vin) {
  __shared__ BatchLds L;
  for (int pi = blockIdx.x; pi < nprob; pi += gridDim.x) {
    const BatchProb& P = probs[pi];
    for (int j = threadIdx.x; j < P.F; j += kBT) L.V[j] = vin[pi][j];
    __syncthreads();
    wg_gram(P, L, P.t);
    __syncthreads();
  }
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// Scratch of the allocation-free persistent solve: descriptors, order,
// records and the queue counter of at most kStaticProblems problems, in one
// file-scope device array per GPU (kept until the process ends).  Host code
// must not pass the array's name to a kernel: it takes the device address
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kStaticProbBytes = (sizeof(BatchProb) * kStaticProblems + 255) / 256 * 256;
constexpr size_t kStaticOrderBytes = (sizeof(int) * kStaticProblems + 255) / 256 * 256;
constexpr size_t kStaticOutBytes = (sizeof(BatchOut) * kStaticProblems + 255) / 256 * 256;
constexpr size_t kStaticScratchBytes = kStaticProbBytes + kStaticOrderBytes + kStaticOutBytes + 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

rr_status batch_scratch(BatchScratch* out) {
  static std::mutex mu;
  static unsigned char* ptrs[64] = {};
  int dev = 0;
  RR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(RR_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    RR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(RR_ERR_DEVICE, "hipGetSymbolAddress returned no address");
    ptrs[dev] = static_cast<unsigned char*>(p);
  }
  unsigned char* base = ptrs[dev];
  out->probs = reinterpret_cast<BatchProb*>(base);
  out->order = reinterpret_cast<int*>(base + kStaticProbBytes);
  out->out = reinterpret_cast<BatchOut*>(base + kStaticProbBytes + kStaticOrderBytes);
  out->queue = reinterpret_cast<int*>(base + kStaticProbBytes + kStaticOrderBytes + kStaticOutBytes);
  out->cap = kStaticProblems;
  return RR_OK;
}

void launch_batch_solve(const BatchProb* probs, const int* order, int nprob, int* queue, BatchOut* out,
                        int grid, hipStream_t s) {
  k_zero_int<<<1, 64, 0, s>>>(queue);
  k_batch_solve<<<grid, kBT, 0, s>>>(probs, order, nprob, queue, out);
}

void launch_batch_gram(const BatchProb* probs, int nprob, const double* const* vin, int grid, hipStream_t s) {
  k_batch_gram<<<grid, kBT, 0, s>>>(probs, nprob, vin);
}

namespace {
// lanes per row of the persistent solve, tuned per shape bucket and device
std::mutex g_btune_mu;
std::map<std::string, int> g_btune;

// Mean time of one operator application of this problem on one workgroup
// (the persistent solve's situation) with `grow` lanes per row.
rr_status time_batch_gram(const BatchPlan& bp, const Sparse& X, int grow, BatchProb* d_prob,
                          const double* const* d_vin, double* t, hipStream_t s, float* ms) {
  BatchProb P;
  std::memset(&P, 0, sizeof(P));
  P.N = X.N;
  P.F = X.F;
  P.nchunk = bp.nchunk;
  P.grow = grow;
  for (int c = 0; c < 3; ++c) P.cls[c] = bp.cls[c];
  P.rp = X.row_ptr;
  P.ci = bp.ci16;
  P.ri = bp.ri16;
  P.csplit = bp.csplit;
  P.t = t;
  RR_HIP(hipMemcpyAsync(d_prob, &P, sizeof(P), hipMemcpyHostToDevice, s));
  hipEvent_t a, b;
  RR_HIP(hipEventCreate(&a));
  RR_HIP(hipEventCreate(&b));
  constexpr int kReps = 3;
  launch_batch_gram(d_prob, 1, d_vin, 1, s);
  RR_HIP(hipEventRecord(a, s));
  for (int i = 0; i < kReps; ++i) launch_batch_gram(d_prob, 1, d_vin, 1, s);
  RR_HIP(hipEventRecord(b, s));
  RR_HIP(hipEventSynchronize(b));
  RR_HIP(hipEventElapsedTime(ms, a, b));
  *ms /= kReps;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return RR_OK;
}
}  // namespace

// Setup of a 0/1 handle with F <= kBatchFMax: the CSC entry offsets of every
// column at every row-chunk boundary and the column classes by length.
// With autotune, the lanes per row come from timing half, once and twice the
// default on one workgroup (cached per shape bucket and device).
rr_status build_batch_plan(BatchPlan& bp, const Sparse& X, hipStream_t s, int autotune) {
  free_batch_plan(bp);
  if (!X.binary || X.F > kBatchFMax || X.F == 0) return RR_OK;
  const int N = X.N, F = X.F;
  std::vector<int> cp(F + 1), ri(std::max(1, X.nnz)), rp(N + 1);
  RR_HIP(hipMemcpyAsync(cp.data(), X.col_ptr, sizeof(int) * (F + 1), hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(rp.data(), X.row_ptr, sizeof(int) * (N + 1), hipMemcpyDeviceToHost, s));
  if (X.nnz) RR_HIP(hipMemcpyAsync(ri.data(), X.row_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  const int nchunk = std::max(1, cdiv(N, kBatchRows));
  std::vector<int> cs((size_t)(nchunk + 1) * F);
  for (int j = 0; j < F; ++j) {
    int k = cp[j];
    for (int h = 0; h <= nchunk; ++h) {
      const long long lim = std::min<long long>((long long)h * kBatchRows, N);
      while (k < cp[j + 1] && ri[k] < lim) ++k;
      cs[(size_t)h * F + j] = (h == nchunk) ? cp[j + 1] : k;
    }
  }
  // classes: 64 lanes from 1024 entries, 16 from 256, 4 from 64, so a lane
  // gets at least 16 entries (one batch of loads); the columns are in
  // descending-count order, so each class is a prefix range
  int cls[3] = {0, 0, 0};
  const int thr[3] = {1024, 256, 64};
  for (int c = 0; c < 3; ++c) {
    int j = c ? cls[c - 1] : 0;
    while (j < F && cp[j + 1] - cp[j] >= thr[c]) ++j;
    cls[c] = j;
  }
  for (int j = 1; j < F; ++j)   // the classes assume the popularity order
    if (cp[j + 1] - cp[j] > cp[j] - cp[j - 1]) return RR_OK;
  const double avg = N > 0 ? (double)X.nnz / N : 0.0;
  int g = 1;
  while (g < 64 && 32.0 * g < avg) g *= 2;   // 16 to 32 entries per lane
  bp.nchunk = nchunk;
  bp.grow = g;
  for (int c = 0; c < 3; ++c) bp.cls[c] = cls[c];
  // 16-bit index copies: column indices (< 8192) and row indices less the
  // first row of their chunk (< 10240), half the index bytes per pass
  const size_t nz = (size_t)std::max(1, X.nnz);
  std::vector<int> ci(nz);
  if (X.nnz) RR_HIP(hipMemcpyAsync(ci.data(), X.col_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  std::vector<uint16_t> c16(nz, 0), r16(nz, 0);
  for (int k = 0; k < X.nnz; ++k) {
    c16[k] = (uint16_t)ci[k];
    r16[k] = (uint16_t)(ri[k] % kBatchRows);
  }
  RR_HIP(dmalloc(&bp.csplit, sizeof(int) * cs.size()));
  RR_HIP(dmalloc(&bp.ci16, sizeof(uint16_t) * nz));
  RR_HIP(dmalloc(&bp.ri16, sizeof(uint16_t) * nz));
  if ((reinterpret_cast<uintptr_t>(bp.ci16) | reinterpret_cast<uintptr_t>(bp.ri16)) % 8)
    return fail(RR_ERR_DEVICE, "internal: index copies not 8-byte aligned");
  RR_HIP(hipMemcpyAsync(bp.csplit, cs.data(), sizeof(int) * cs.size(), hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(bp.ci16, c16.data(), sizeof(uint16_t) * nz, hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(bp.ri16, r16.data(), sizeof(uint16_t) * nz, hipMemcpyHostToDevice, s));
  RR_HIP(hipStreamSynchronize(s));
  if (!autotune || X.nnz == 0) return RR_OK;
  int dev = 0;
  RR_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  RR_HIP(hipGetDeviceProperties(&prop, dev));
  auto lg = [](long long v) { int b = 0; while ((1LL << b) < v) ++b; return b; };
  const std::string key = std::string(prop.gcnArchName) + ":" + std::to_string(lg(N)) + ":" +
                          std::to_string(lg(F)) + ":" + std::to_string(lg(X.nnz));
  {
    std::lock_guard<std::mutex> lk(g_btune_mu);
    auto it = g_btune.find(key);
    if (it != g_btune.end()) {
      bp.grow = it->second;
      bp.tuned = 2;
      return RR_OK;
    }
  }
  BatchProb* d_prob = nullptr;
  double *v = nullptr, *t = nullptr;
  const double** d_vin = nullptr;
  rr_status st = RR_OK;
  if (dmalloc(&d_prob, sizeof(BatchProb)) != hipSuccess || dmalloc(&v, sizeof(double) * F) != hipSuccess ||
      dmalloc(&t, sizeof(double) * F) != hipSuccess || dmalloc(&d_vin, sizeof(double*)) != hipSuccess)
    st = fail(RR_ERR_DEVICE, "out of device memory for the batched plan's tuning");
  if (st == RR_OK) {
    launch_fill(v, 1.0, F, s);
    const double* hv = v;
    if (hipMemcpyAsync(d_vin, &hv, sizeof(double*), hipMemcpyHostToDevice, s) != hipSuccess)
      st = fail(RR_ERR_DEVICE, "tuning copy failed");
  }
  int best = g;
  float best_ms = 1e30f;
  for (int cand : {g, std::max(1, g / 2), std::min(64, 2 * g)}) {
    if (st != RR_OK) break;
    float ms = 0.f;
    st = time_batch_gram(bp, X, cand, d_prob, d_vin, t, s, &ms);
    // another value must win by 3 % over the default
    if (st == RR_OK && (cand == g ? ms < best_ms : ms < 0.97f * best_ms)) {
      best_ms = ms;
      best = cand;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)dev_free(d_prob);
  (void)dev_free(v);
  (void)dev_free(t);
  (void)dev_free(d_vin);
  RR_TRY(st);
  bp.grow = best;
  bp.tuned = 1;
  std::lock_guard<std::mutex> lk(g_btune_mu);
  g_btune[key] = best;
  return RR_OK;
}

void free_batch_plan(BatchPlan& bp) {
  if (bp.csplit) (void)dev_free(bp.csplit);
  if (bp.ci16) (void)dev_free(bp.ci16);
  if (bp.ri16) (void)dev_free(bp.ri16);
  bp = BatchPlan{};
}

}  // namespace rr
