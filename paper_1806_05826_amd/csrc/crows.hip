// u2 = u1 + S (s o yc) for the second operator application of the V(1,1)
// cycle of the two-level-iteration subsection (0/1 X).  The cycle applies A
// to e1 and then to e2 = e1 + P yc, with (P yc)_j = s_l(j) yc_l(j) (the
// adjusted square-root-average prolongation of the data-matrices
// subsection, s_c = 1/sqrt(n_c)).  Since X e2 = X e1 + X P yc and X P yc gathers, for
// every row, s_l yc_l over the labels l of its entries, the row pass of e2
// reduces to u1 = X e1 (already formed) plus a gather from an F_C-entry
// vector that fits in LDS whole: no slices, no partial sums, no reduction.
// The table holds X's pattern with every column index replaced by its
// cluster label, in layers of 64 rows of nearly equal length (entry k of
// lane l at base + 256 (k / 4) + 4 l + k % 4, padded with label F_C, whose
// LDS entry is zero); each wave adds one layer's 64 rows.
#include <algorithm>
#include <numeric>
#include <vector>

#include "rr_device.h"

namespace rr {

namespace {

constexpr int kCrThreads = 256;
constexpr int kCrUnroll = 16;   // 8-byte label loads in flight per lane (64 entries)

// One wave per layer: its descriptor, row ids, u1 and first 16 label loads
// are issued before the workgroup fills the LDS vector.  T is the type of u
// and of the sums (FP64, or FP32 for the single-precision inner solves,
// whose prolongation rounds s_l yc_l to FP32 the same way).
template <typename T>
__global__ __launch_bounds__(kCrThreads) void k_cluster_rows(int nlayer, const int2* __restrict__ layer,
                                                             const uint16_t* __restrict__ ent,
                                                             const int* __restrict__ rowid, int FC,
                                                             const double* __restrict__ cscale,
                                                             const double* __restrict__ yc,
                                                             const double* __restrict__ rw,
                                                             T* __restrict__ u, const int* done) {
  extern __shared__ __align__(8) unsigned char yt_raw[];
  T* yt = reinterpret_cast<T*>(yt_raw);   // [FC + 1]
  if (is_done(done)) return;
  const int lane = threadIdx.x & 63;
  const int L = blockIdx.x * (kCrThreads / 64) + (threadIdx.x >> 6);
  const bool active = L < nlayer;
  const int2 d = active ? layer[L] : make_int2(0, 0);   // (first entry, entries per lane)
  const int row = active ? rowid[(size_t)L * 64 + lane] : -1;
  const T u0 = row >= 0 ? u[row] : T(0);
  const uint2* p = reinterpret_cast<const uint2*>(ent + d.x) + lane;
  const int ng = d.y / 4;
  uint2 q[kCrUnroll];
#pragma unroll
  for (int j = 0; j < kCrUnroll; ++j) q[j] = (j < ng) ? p[(size_t)j * 64] : make_uint2(0u, 0u);
  for (int c = threadIdx.x; c <= FC; c += kCrThreads) yt[c] = c < FC ? (T)(cscale[c] * yc[c]) : T(0);
  __syncthreads();
  T acc = T(0);
  for (int g = 0; g < ng; g += kCrUnroll) {
    if (g > 0) {
#pragma unroll
      for (int j = 0; j < kCrUnroll; ++j) q[j] = (g + j < ng) ? p[(size_t)(g + j) * 64] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < kCrUnroll; ++j) {
      if (g + j < ng) {
        acc += yt[q[j].x & 0xffffu];
        acc += yt[q[j].x >> 16];
        acc += yt[q[j].y & 0xffffu];
        acc += yt[q[j].y >> 16];
      }
    }
  }
  if (row >= 0) u[row] = rw ? u0 + (T)rw[row] * acc : u0 + acc;   // D X P yc with row weights
}

}  // namespace

namespace {

// Xc[c][i] = s_c sqrt(d_i) (count of label c in row i): the columns of
// D^1/2 X P as rows, from the label table; each lane owns its row, so the
// additions are plain and in a fixed order.
__global__ __launch_bounds__(kCrThreads) void k_weighted_xc(int nlayer, const int2* __restrict__ layer,
                                                            const uint16_t* __restrict__ ent,
                                                            const int* __restrict__ rowid, int FC, int Np,
                                                            const double* __restrict__ cscale,
                                                            const double* __restrict__ rw, double* Xc) {
  const int lane = threadIdx.x & 63;
  const int L = blockIdx.x * (kCrThreads / 64) + (threadIdx.x >> 6);
  if (L >= nlayer) return;
  const int2 d = layer[L];
  const int row = rowid[(size_t)L * 64 + lane];
  if (row < 0) return;
  const double sd = sqrt(rw[row]);
  for (int k = 0; k < d.y; ++k) {
    const int c = ent[(size_t)d.x + (size_t)(k / 4) * 256 + (size_t)lane * 4 + k % 4];
    if (c < FC) Xc[(size_t)c * Np + row] += cscale[c] * sd;
  }
}

}  // namespace

// K = P^T X^T D X P = (D^1/2 X P)^T (D^1/2 X P) in one pass over the label
// table and one FP64 GEMM (setup of row weights).
rr_status weighted_gram_from_labels(rr_handle* h, hipStream_t s) {
  const ClusterRows& cr = h->crow;
  const int FC = h->FC, N = h->X.N;
  const int FCp = (FC + 127) / 128 * 128, Np = (N + 127) / 128 * 128;
  const size_t bytes = sizeof(double) * (size_t)FCp * Np;
  if (!h->wxc) RR_HIP(dmalloc(&h->wxc, bytes));
  RR_HIP(hipMemsetAsync(h->wxc, 0, bytes, s));
  k_weighted_xc<<<cdiv(cr.nlayer, kCrThreads / 64), kCrThreads, 0, s>>>(cr.nlayer, cr.layer, cr.ent, cr.rowid,
                                                                        FC, Np, h->cscale, h->X.rw, h->wxc);
  return gram_rows(h->wxc, FC, FCp, Np, h->K, s);
}

void free_cluster_rows(ClusterRows& cr) {
  if (cr.layer) (void)dev_free(cr.layer);
  if (cr.ent) (void)dev_free(cr.ent);
  if (cr.rowid) (void)dev_free(cr.rowid);
  cr = ClusterRows{};
}

// Setup only: the label table of X's rows (0/1 X, F_C <= kMaxCrClusters).
rr_status build_cluster_rows(rr_handle* h, hipStream_t s) {
  ClusterRows& cr = h->crow;
  free_cluster_rows(cr);
  free_sell(h->xp);
  free_merge_plan(h->xp_restrict);
  const Sparse& X = h->X;
  const int N = X.N, F = X.F, FC = h->FC;
  if (!X.binary || FC < 1 || FC > kMaxCrClusters || N < 1) return RR_OK;
  std::vector<int> rp(N + 1), ci(std::max(1, X.nnz)), lab(F);
  RR_HIP(hipMemcpyAsync(rp.data(), X.row_ptr, sizeof(int) * (N + 1), hipMemcpyDeviceToHost, s));
  if (X.nnz) RR_HIP(hipMemcpyAsync(ci.data(), X.col_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(lab.data(), h->labels, sizeof(int) * F, hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  // rows, longest first (ties in row order), 64 to a layer
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
  const int nlayer = cdiv(N, 64);
  std::vector<int2> layer(nlayer);
  std::vector<int> rowid((size_t)nlayer * 64, -1);
  size_t total = 0;
  for (int L = 0; L < nlayer; ++L) {
    const int r0 = order[(size_t)L * 64];
    const int len = ((rp[r0 + 1] - rp[r0]) + 3) / 4 * 4;
    if (total + (size_t)std::max(len, 4) * 64 >= (size_t)INT32_MAX) return RR_OK;   // table too large
    layer[L] = make_int2((int)total, std::max(len, 4));
    total += (size_t)std::max(len, 4) * 64;
  }
  std::vector<uint16_t> ent(total, (uint16_t)FC);
  for (int L = 0; L < nlayer; ++L) {
    for (int l = 0; l < 64; ++l) {
      const size_t i = (size_t)L * 64 + l;
      if (i >= (size_t)N) break;
      const int r = order[i];
      rowid[i] = r;
      for (int k = 0, e = rp[r]; e < rp[r + 1]; ++k, ++e) {
        const int c = lab[ci[e]];
        if (c < 0 || c >= FC) return fail(RR_ERR_DEVICE, "internal: label out of range");
        ent[(size_t)layer[L].x + (size_t)(k / 4) * 256 + (size_t)l * 4 + k % 4] = (uint16_t)c;
      }
    }
  }
  RR_HIP(dmalloc(&cr.layer, sizeof(int2) * nlayer));
  RR_HIP(dmalloc(&cr.ent, sizeof(uint16_t) * total));
  RR_HIP(dmalloc(&cr.rowid, sizeof(int) * rowid.size()));
  RR_HIP(hipMemcpyAsync(cr.layer, layer.data(), sizeof(int2) * nlayer, hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(cr.ent, ent.data(), sizeof(uint16_t) * total, hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(cr.rowid, rowid.data(), sizeof(int) * rowid.size(), hipMemcpyHostToDevice, s));
  RR_HIP(hipStreamSynchronize(s));
  cr.nlayer = nlayer;
  // the column pass of X P, for the V(1,1) restriction from the row pass
  // (only where the restriction's finishing step fits the coarse GEMV)
  if (X.sliced && restrict_gemv_fusable(h->restrict_plan, FC)) {
    RR_TRY(build_xp_plan(h->xp, rp, ci, lab, N, FC, X.num_cu, h->tuning.div_cols, s));
    RR_TRY(build_xp_restrict(h->xp_restrict, h->xp, h->coff, FC, F, s));
  }
  return RR_OK;
}

void launch_cluster_rows(const rr_handle* h, const double* yc, const double* rw, double* u, const int* done,
                         hipStream_t s) {
  const ClusterRows& cr = h->crow;
  const int g = cdiv(cr.nlayer, kCrThreads / 64);
  k_cluster_rows<double><<<g, kCrThreads, sizeof(double) * (h->FC + 1), s>>>(
      cr.nlayer, cr.layer, cr.ent, cr.rowid, h->FC, h->cscale, yc, rw, u, done);
}

void launch_cluster_rows32(const rr_handle* h, const double* yc, float* u, const int* done, hipStream_t s) {
  const ClusterRows& cr = h->crow;
  const int g = cdiv(cr.nlayer, kCrThreads / 64);
  k_cluster_rows<float><<<g, kCrThreads, sizeof(float) * (h->FC + 1), s>>>(
      cr.nlayer, cr.layer, cr.ent, cr.rowid, h->FC, h->cscale, yc, nullptr, u, done);
}

}  // namespace rr
