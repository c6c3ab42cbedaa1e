// The cluster-aligned block smoother of the two-level cycle: S = omega D_B^-1,
// D_B the block diagonal of A = X^T X + lam I over blocks of at most 32
// features inside one cluster (each cluster's features in increasing caller
// index, cut into consecutive groups).  The blocks' Gram matrices X_B^T X_B
// are formed once at setup (exact integers for 0/1 X); each lambda gets the
// explicit inverses (X_B^T X_B + lam I)^-1, 32 x 32 per block.
#include <algorithm>
#include <vector>

#include "rr_device.h"

namespace rr {

namespace {

constexpr int kB = kSmoothBlock;           // 32
constexpr int kBB = kSmoothBlock * kSmoothBlock;

// G_b[i][k] += x_ri x_rk for every row r and pair of its entries (i, k) in
// one block; one thread per row.  0/1 X counts in exact integers.
__global__ void k_block_gram_bin(int N, const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                 const int* __restrict__ bid, const int* __restrict__ bloc,
                                 unsigned* __restrict__ G) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= N) return;
  const int a = row_ptr[row], e = row_ptr[row + 1];
  for (int p = a; p < e; ++p) {
    const int j = col_idx[p];
    const int bj = bid[j], lj = bloc[j];
    for (int q = p; q < e; ++q) {
      const int k = col_idx[q];
      if (bid[k] != bj) continue;
      const int lk = bloc[k];
      atomicAdd(&G[(size_t)bj * kBB + lj * kB + lk], 1u);
      if (q != p) atomicAdd(&G[(size_t)bj * kBB + lk * kB + lj], 1u);
    }
  }
}

__global__ void k_block_gram_val(int N, const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                                 const double* __restrict__ val, const int* __restrict__ bid,
                                 const int* __restrict__ bloc, double* __restrict__ G) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= N) return;
  const int a = row_ptr[row], e = row_ptr[row + 1];
  for (int p = a; p < e; ++p) {
    const int j = col_idx[p];
    const int bj = bid[j], lj = bloc[j];
    for (int q = p; q < e; ++q) {
      const int k = col_idx[q];
      if (bid[k] != bj) continue;
      const int lk = bloc[k];
      const double v = val[p] * val[q];
      atomicAdd(&G[(size_t)bj * kBB + lj * kB + lk], v);
      if (q != p) atomicAdd(&G[(size_t)bj * kBB + lk * kB + lj], v);
    }
  }
}

__global__ void k_u32_to_f64(long long n, const unsigned* a, double* b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// One wave per block: (G_b + lam I)^-1 by Gauss-Jordan on [A | I] in LDS
// (A is SPD, so no pivoting is needed); lane c owns column c of the 32 x 64
// augmented matrix.  A non-positive pivot sets *bad.
__global__ __launch_bounds__(64) void k_block_inv(const int* __restrict__ boff, const double* __restrict__ G,
                                                  double lam, double* __restrict__ Dinv, int* bad) {
  const int b = blockIdx.x;
  const int n = boff[b + 1] - boff[b];
  const int c = threadIdx.x;
  __shared__ double M[kB][2 * kB + 1];
  __shared__ double colk[kB];
  const double* g = G + (size_t)b * kBB;
  for (int i = 0; i < kB; ++i) {
    double v;
    if (c < kB) v = (i < n && c < n) ? g[i * kB + c] + (i == c ? lam : 0.0) : (i == c ? 1.0 : 0.0);
    else v = (i == c - kB) ? 1.0 : 0.0;
    M[i][c] = v;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = M[k][k];
    if (!(piv > 0.0)) {
      if (c == 0) *bad = 1;
      return;
    }
    if (c < kB) colk[c] = M[c][k];
    __syncthreads();
    M[k][c] = M[k][c] / piv;
    __syncthreads();
    for (int i = 0; i < n; ++i)
      if (i != k) M[i][c] -= colk[i] * M[k][c];
    __syncthreads();
  }
  double* d = Dinv + (size_t)b * kBB;
  if (c < kB)
    for (int i = 0; i < kB; ++i) d[i * kB + c] = (i < n && c < n) ? M[i][kB + c] : 0.0;
}

// out_j = base_j + omega (D_B^-1 rho)_j + (P yc)_j over the features of
// every block (base, yc optional); 8 blocks per 256-thread workgroup, one
// per 32-lane half-wave (lane i forms row i of its block); with parts, one
// <r, out> partial per workgroup.
constexpr int kSmoothThreads = 256;
__global__ __launch_bounds__(kSmoothThreads) void k_block_smooth(
    int nblk, const int* __restrict__ boff, const int* __restrict__ bperm, const double* __restrict__ Dinv,
    double omega, const double* __restrict__ rho, const double* __restrict__ base,
    const int* __restrict__ labels, const double* __restrict__ cscale, const double* __restrict__ yc,
    const double* __restrict__ r, double* __restrict__ out, double* parts, const int* done) {
  if (is_done(done)) return;
  const int half = threadIdx.x >> 5, hl = threadIdx.x & 31;
  double dot = 0.0;
  for (int b = blockIdx.x * (kSmoothThreads / 32) + half; b < nblk; b += gridDim.x * (kSmoothThreads / 32)) {
    const int o = boff[b], n = boff[b + 1] - o;
    const int j = hl < n ? bperm[o + hl] : -1;
    const double rv = j >= 0 ? rho[j] : 0.0;
    const double* drow = Dinv + (size_t)b * kBB + hl * kB;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += drow[k] * __shfl(rv, k, 32);
    if (j >= 0) {
      double v = omega * acc;
      if (base) v += base[j];
      if (yc) {
        const int l = labels[j];
        v += cscale[l] * yc[l];
      }
      out[j] = v;
      if (parts) dot += r[j] * v;
    }
  }
  if (parts) store_block_partial<kSmoothThreads>(dot, parts, blockIdx.x);
}

}  // namespace

// Blocks from the aggregation (labels, caller order through fperm) and their
// Gram matrices.  Setup only.
rr_status build_smoother_blocks(rr_handle* h, hipStream_t s) {
  const Sparse& X = h->X;
  const int F = X.F, FC = h->FC;
  std::vector<int> lab(F), fperm(F);
  RR_HIP(hipMemcpyAsync(lab.data(), h->labels, sizeof(int) * F, hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(fperm.data(), h->fperm, sizeof(int) * F, hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  // members of each cluster in increasing caller index
  std::vector<std::vector<int>> mem(FC);
  std::vector<int> order(F);
  for (int j = 0; j < F; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return fperm[a] < fperm[b]; });
  for (int j : order) {
    if (lab[j] < 0 || lab[j] >= FC) return fail(RR_ERR_DEVICE, "internal: label out of range");
    mem[lab[j]].push_back(j);
  }
  std::vector<int> boff{0}, bperm, bid(F), bloc(F);
  for (int c = 0; c < FC; ++c)
    for (size_t a = 0; a < mem[c].size(); a += kB) {
      const int blk = (int)boff.size() - 1;
      const size_t e = std::min(mem[c].size(), a + kB);
      for (size_t i = a; i < e; ++i) {
        bid[mem[c][i]] = blk;
        bloc[mem[c][i]] = (int)(i - a);
        bperm.push_back(mem[c][i]);
      }
      boff.push_back((int)bperm.size());
    }
  if ((int)bperm.size() != F) return fail(RR_ERR_DEVICE, "internal: smoother blocks miss a feature");
  const int nblk = (int)boff.size() - 1;
  int *d_bid = nullptr, *d_bloc = nullptr;
  RR_HIP(dmalloc(&h->boff, sizeof(int) * (nblk + 1)));
  RR_HIP(dmalloc(&h->bperm, sizeof(int) * F));
  RR_HIP(dmalloc(&d_bid, sizeof(int) * F));
  RR_HIP(dmalloc(&d_bloc, sizeof(int) * F));
  RR_HIP(dmalloc(&h->bgram, sizeof(double) * (size_t)nblk * kBB));
  RR_HIP(hipMemcpyAsync(h->boff, boff.data(), sizeof(int) * (nblk + 1), hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(h->bperm, bperm.data(), sizeof(int) * F, hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(d_bid, bid.data(), sizeof(int) * F, hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(d_bloc, bloc.data(), sizeof(int) * F, hipMemcpyHostToDevice, s));
  const long long nn = (long long)nblk * kBB;
  if (X.binary) {
    unsigned* Gi = nullptr;
    RR_HIP(dmalloc(&Gi, sizeof(unsigned) * nn));
    RR_HIP(hipMemsetAsync(Gi, 0, sizeof(unsigned) * nn, s));
    k_block_gram_bin<<<cdiv(X.N, kBlock), kBlock, 0, s>>>(X.N, X.row_ptr, X.col_idx, d_bid, d_bloc, Gi);
    k_u32_to_f64<<<cdiv(nn, kBlock), kBlock, 0, s>>>(nn, Gi, h->bgram);
    RR_HIP(hipStreamSynchronize(s));
    RR_HIP(dev_free(Gi));
  } else {
    RR_HIP(hipMemsetAsync(h->bgram, 0, sizeof(double) * nn, s));
    k_block_gram_val<<<cdiv(X.N, kBlock), kBlock, 0, s>>>(X.N, X.row_ptr, X.col_idx, X.val, d_bid, d_bloc,
                                                          h->bgram);
  }
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  RR_HIP(dev_free(d_bid));
  RR_HIP(dev_free(d_bloc));
  h->nblk = nblk;
  return RR_OK;
}

rr_status block_factor(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s) {
  if (h->nblk == 0) return RR_OK;
  if (!slot.Dinv) RR_HIP(dmalloc(&slot.Dinv, sizeof(double) * (size_t)h->nblk * kBB));
  RR_HIP(hipMemsetAsync(h->chol_flag, 0, sizeof(int), s));
  k_block_inv<<<h->nblk, 64, 0, s>>>(h->boff, h->bgram, lam, slot.Dinv, h->chol_flag);
  int bad = 0;
  RR_HIP(hipMemcpyAsync(&bad, h->chol_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  if (bad) return fail(RR_ERR_BREAKDOWN, "a smoother block is not numerically positive definite");
  slot.omega_block = 0.0;
  return RR_OK;
}

int launch_block_smooth(const rr_handle* h, const double* Dinv, double omega, const double* rho,
                        const double* base, const double* yc, const double* r, double* out,
                        double* parts, const int* done, hipStream_t s) {
  const int g = std::max(1, std::min(cdiv(h->nblk, kSmoothThreads / 32), 512));
  k_block_smooth<<<g, kSmoothThreads, 0, s>>>(h->nblk, h->boff, h->bperm, Dinv, omega, rho, base,
                                              h->labels, h->cscale, yc, r, out, parts, done);
  return g;
}

}  // namespace rr
