// The matrix-free operator v -> X^T (X v) + lambda v as two sparse passes:
//   u = X v     CSR, a fixed group of lanes per row (rows are short and even)
//   t = X^T u   CSC, merge-path tiles over (column ends + nonzeros), so the
//               Zipf-skewed column lengths cost the same per tile; columns
//               that cross tiles are finished by a small fix-up kernel that
//               adds the tile partials in tile order (deterministic).
// Only the matrix-vector product is needed by the Krylov method (the paper's
// introduction); X^T X is never formed.
#include <climits>

#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "rr_device.h"

namespace rr {

// ---------------------------------------------------------------------------
// CSR: u[i] = sum_{e in row i} v[col[e]] (* val[e])
// ---------------------------------------------------------------------------
template <int G, bool BIN>
__global__ __launch_bounds__(kBlock) void k_csr(const int* __restrict__ ptr,
                                                const int* __restrict__ idx,
                                                const double* __restrict__ val,
                                                const double* __restrict__ v,
                                                double* __restrict__ u, int nrows,
                                                const int* done) {
  if (is_done(done)) return;
  const int lane = threadIdx.x & (G - 1);
  const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
  if (row >= nrows) return;  // whole G-lane group leaves together
  const int a = ptr[row], b = ptr[row + 1];
  double acc0 = 0.0, acc1 = 0.0;
  int e = a + lane;
  for (; e + G < b; e += 2 * G) {
    const int c0 = idx[e], c1 = idx[e + G];
    double x0 = v[c0], x1 = v[c1];
    if (!BIN) {
      x0 *= val[e];
      x1 *= val[e + G];
    }
    acc0 += x0;
    acc1 += x1;
  }
  if (e < b) {
    double x0 = v[idx[e]];
    if (!BIN) x0 *= val[e];
    acc0 += x0;
  }
  double acc = acc0 + acc1;
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  if (lane == 0) u[row] = acc;
}

template <int G>
static void csr_dispatch(const Sparse& X, const double* v, double* u, const int* done,
                         hipStream_t s) {
  const int grid = cdiv((long long)X.N * G, kBlock);
  if (X.binary)
    k_csr<G, true><<<grid, kBlock, 0, s>>>(X.row_ptr, X.col_idx, nullptr, v, u, X.N, done);
  else
    k_csr<G, false><<<grid, kBlock, 0, s>>>(X.row_ptr, X.col_idx, X.val, v, u, X.N, done);
}

void launch_csr(const Sparse& X, const double* v, double* u, const int* done, hipStream_t s,
                const StageArgs* stage, hipEvent_t mid) {
  if (X.sliced && X.N > 0) {
    // u = D X v with row weights, applied as each row is finished
    launch_rows(X.rows, v, u, X.rw, done, s, stage);
    if (mid) (void)hipEventRecord(mid, s);
    return;
  }
  if (stage) launch_stage_update(*stage, s);
  if (X.N == 0) {
    if (mid) (void)hipEventRecord(mid, s);
    return;
  }
  switch (X.csr_group) {
    case 4: csr_dispatch<4>(X, v, u, done, s); break;
    case 8: csr_dispatch<8>(X, v, u, done, s); break;
    case 16: csr_dispatch<16>(X, v, u, done, s); break;
    case 32: csr_dispatch<32>(X, v, u, done, s); break;
    default: csr_dispatch<64>(X, v, u, done, s); break;
  }
  if (X.rw) launch_row_scale(X.N, X.rw, u, u, s);
  if (mid) (void)hipEventRecord(mid, s);
}

bool csr_pupd_ok(const Sparse& X) { return X.sliced && X.N > 0 && X.rows.nblk > 0 && !X.rows.hval; }

void launch_csr_pupd(const Sparse& X, const double* z, double* up, const int* done, hipStream_t s,
                     const PUpd& pu, hipEvent_t mid) {
  launch_rows_pupd(X.rows, z, up, X.rw, done, s, pu);
  if (mid) (void)hipEventRecord(mid, s);
}

// ---------------------------------------------------------------------------
// Merge-path segmented gather-sum.  The merged list holds, for every
// segment, its nonzeros followed by an end marker.  Tile b covers merged
// items [b*T, (b+1)*T); coord[b] = (segments ended before, nonzeros before).
// ---------------------------------------------------------------------------
__device__ inline int merge_search(int diag, int alen, int blen, const int* a_end) {
  // number of segment ends among the first `diag` merged items
  int lo = max(0, diag - blen), hi = min(diag, alen);
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (a_end[m] <= diag - m - 1)
      lo = m + 1;
    else
      hi = m;
  }
  return lo;
}

__global__ void k_merge_coord(const int* __restrict__ seg_end, int nseg, int nnz,
                              int nblocks, int2* __restrict__ coord) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblocks) return;
  const long long total = (long long)nseg + nnz;
  const int diag = (int)min((long long)b * kMergeTile, total);
  const int x = merge_search(diag, nseg, nnz, seg_end);
  coord[b] = make_int2(x, diag - x);
}

template <int MODE, bool BIN>
__global__ __launch_bounds__(kBlock) void k_segsum(
    const int* __restrict__ seg_end, const int* __restrict__ idx,
    const double* __restrict__ val, const double* __restrict__ v,
    const int2* __restrict__ coord, double* __restrict__ head, double* __restrict__ tail,
    int nseg, int nslots, Epi e, const int* done) {
  if (is_done(done)) return;
  __shared__ int s_end[kMergeTile + 1];
  __shared__ double s_val[kMergeTile];
  __shared__ int s_flag[kBlock];
  __shared__ double s_acc[kBlock];

  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int2 c0 = coord[b], c1 = coord[b + 1];
  const int x0 = c0.x, y0 = c0.y;
  const int nx = c1.x - x0, ny = c1.y - y0;
  const int total = nx + ny;

  {
    // issue all staging loads before the first LDS store
    int te[kMergeItems + 1];
    int ti[kMergeItems];
#pragma unroll
    for (int k = 0; k <= kMergeItems; ++k) {
      const int i = tid + k * kBlock;
      te[k] = (i <= nx && x0 + i < nseg) ? seg_end[x0 + i] - y0 : INT_MAX;
    }
#pragma unroll
    for (int k = 0; k < kMergeItems; ++k) {
      const int i = tid + k * kBlock;
      ti[k] = (i < ny) ? idx[y0 + i] : 0;
    }
    double tv[kMergeItems];
#pragma unroll
    for (int k = 0; k < kMergeItems; ++k) {
      const int i = tid + k * kBlock;
      double a = 0.0;
      if (i < ny) {
        a = v[ti[k]];
        if (!BIN) a *= val[y0 + i];
      }
      tv[k] = a;
    }
#pragma unroll
    for (int k = 0; k <= kMergeItems; ++k) {
      const int i = tid + k * kBlock;
      if (i <= nx) s_end[i] = te[k];
    }
#pragma unroll
    for (int k = 0; k < kMergeItems; ++k) {
      const int i = tid + k * kBlock;
      if (i < ny) s_val[i] = tv[k];
    }
  }
  __syncthreads();

  const int d = min(tid * kMergeItems, total);
  const int dend = min(d + kMergeItems, total);
  const int x = merge_search(d, nx, ny, s_end);
  const int y = d - x;

  // pass 1: the partial sum of the segment this thread's range ends in
  double acc = 0.0;
  int saw = 0;
  {
    int xx = x, yy = y;
#pragma unroll
    for (int k = 0; k < kMergeItems; ++k) {
      if (d + k < dend) {
        if (yy < s_end[xx]) {
          acc += s_val[yy];
          ++yy;
        } else {
          acc = 0.0;
          saw = 1;
          ++xx;
        }
      }
    }
  }
  // segmented inclusive scan over threads: (f1,v1) + (f2,v2) = (f1|f2, f2 ? v2 : v1+v2)
  s_flag[tid] = saw;
  s_acc[tid] = acc;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    int f = s_flag[tid];
    double vv = s_acc[tid];
    if (tid >= off) {
      if (!f) vv = s_acc[tid - off] + vv;
      f |= s_flag[tid - off];
    }
    __syncthreads();
    s_flag[tid] = f;
    s_acc[tid] = vv;
    __syncthreads();
  }
  const double carry = tid ? s_acc[tid - 1] : 0.0;

  // pass 2: finish every segment whose end marker lies in this thread's range
  const int seg_start0 = (x0 > 0) ? seg_end[x0 - 1] : 0;
  const bool mid = seg_start0 < y0;   // tile begins inside segment x0
  double dot = 0.0;
  acc = carry;
  {
    int xx = x, yy = y;
#pragma unroll
    for (int k = 0; k < kMergeItems; ++k) {
      if (d + k < dend) {
        if (yy < s_end[xx]) {
          acc += s_val[yy];
          ++yy;
        } else {
          if (xx == 0 && mid)
            head[b] = acc;
          else
            seg_finish<MODE>(x0 + xx, acc, e, dot);
          acc = 0.0;
          ++xx;
        }
      }
    }
  }
  if (d < dend && dend == total) tail[b] = acc;
  if constexpr (has_dot<MODE>()) {
    double vv[1] = {dot};
    store_block_partial<kBlock>(vv[0], e.partials, b);
  }
}

// One wave per tile-crossing segment: lanes add the tile partials in a fixed
// strided pattern, then a fixed butterfly; head of the last tile added last.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_segfix(const int4* __restrict__ span, int nspan,
                                                   const double* __restrict__ head,
                                                   const double* __restrict__ tail,
                                                   int nmain, Epi e, const int* done) {
  if (is_done(done)) return;
  const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double dot = 0.0;
  if (wave < nspan) {
    const int4 sp = span[wave];
    double acc = 0.0;
    for (int bb = sp.y + lane; bb < sp.z; bb += 64) acc += tail[bb];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    acc += head[sp.z];
    if (lane == 0) seg_finish<MODE>(sp.x, acc, e, dot);
  }
  if constexpr (has_dot<MODE>()) store_block_partial<kBlock>(dot, e.partials, nmain + blockIdx.x);
}

// Segmented sums for epilogues without a dot product (the restriction): a
// segment of at most kWaveSeg entries is one wave's item (lane l adds
// entries l, l + 64, ... in order, 16 loads in flight, then a fixed
// butterfly) and is finished in place; a longer one is cut into chunks of at
// most kWaveSeg entries, each a wave item whose sum goes to cpart, and one
// more wave per such segment (second kernel) adds its chunk sums in chunk
// order and finishes it.  Entry q is v[idx[q]], or v[q] when v is already in
// segment order (IDX false: one load, coalesced).
// XP (with IDX, the plan of build_xp_restrict): entry q is r[j] - lam e1[j]
// (Epi r, p, lam; j = idx[q]); an item that finishes cluster s subtracts the
// sum of its X P column-pass pieces (at most kXpPieces, loaded ahead of the
// entries), and a piece item (x = -1 - s) stores minus the sum of pieces
// [y, z) (at most 512) in its chunk slot, so that cluster s gets
// (P^T (r - lam e1) - (X P)^T u)_s / P_js = (P^T (r - A e1))_s / P_js with
// u = X e1.  Pieces are added lane-strided, then by the fixed butterfly.
constexpr int kWaveSeg = 1024;
constexpr int kSegBlock = 256;
constexpr int kXpPieces = 128;       // pieces a finishing item adds itself
constexpr int kXpPieceItem = 512;    // pieces of one piece item


template <int MODE, bool VAL, bool IDX, bool XP = false>
__global__ __launch_bounds__(kSegBlock) void k_seg1(const int4* __restrict__ witem, int nw,
                                                    const int* __restrict__ idx,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ v, Epi e,
                                                    double* __restrict__ cpart, const int* done) {
  static_assert(!XP || (IDX && !VAL), "the X P form gathers r and e1 through the cluster order");
  if (is_done(done)) return;
  constexpr int U = 16;
  static_assert(U * 64 == kWaveSeg, "a wave item is at most one batch per lane");
  const int wv = (int)blockIdx.x * (kSegBlock / 64) + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wv >= nw) return;
  const int4 it = witem[wv];
  if constexpr (XP) {
    if (it.x < 0) {   // piece item (wave-uniform)
      constexpr int M = kXpPieceItem / 64;
      int pp[M];
      double pv[M];
#pragma unroll
      for (int m = 0; m < M; ++m) pp[m] = it.y + lane + 64 * m < it.z ? e.xpos[it.y + lane + 64 * m] : -1;
#pragma unroll
      for (int m = 0; m < M; ++m) pv[m] = pp[m] >= 0 ? e.xpart[pp[m]] : 0.0;
      double c = 0.0;
#pragma unroll
      for (int m = 0; m < M; ++m) c += pv[m];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
      if (lane == 0) cpart[it.w] = -c;
      return;
    }
  }
  int j[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const int q = it.y + lane + 64 * k;
    j[k] = q < it.z ? (IDX ? idx[q] : q) : -1;
  }
  constexpr int XM = kXpPieces / 64;
  double xv[XM];
#pragma unroll
  for (int m = 0; m < XM; ++m) xv[m] = 0.0;
  if constexpr (XP) {
    if (it.w < 0) {   // this item finishes its cluster (wave-uniform)
      const int q0 = e.xbase[it.x], q1 = e.xbase[it.x + 1];
      int pp[XM];
#pragma unroll
      for (int m = 0; m < XM; ++m) pp[m] = q0 + lane + 64 * m < q1 ? e.xpos[q0 + lane + 64 * m] : -1;
#pragma unroll
      for (int m = 0; m < XM; ++m) xv[m] = pp[m] >= 0 ? e.xpart[pp[m]] : 0.0;
    }
  }
  double t = 0.0;
  if constexpr (XP) {
    double a[U], b[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      a[k] = j[k] >= 0 ? e.r[j[k]] : 0.0;
      b[k] = j[k] >= 0 ? e.p[j[k]] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) t += a[k] - e.lam * b[k];
  } else if constexpr (VAL) {
    double a[U];
#pragma unroll
    for (int k = 0; k < U; ++k) a[k] = j[k] >= 0 ? val[it.y + lane + 64 * k] : 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k) t += j[k] >= 0 ? v[j[k]] * a[k] : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < U; ++k) t += j[k] >= 0 ? v[j[k]] : 0.0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if constexpr (XP) {
    if (it.w < 0) {
      double c = 0.0;
#pragma unroll
      for (int m = 0; m < XM; ++m) c += xv[m];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
      t -= c;
    }
  }
  if (lane == 0) {
    if (it.w < 0) {
      double dot = 0.0;
      seg_finish<MODE>(it.x, t, e, dot);
    } else {
      cpart[it.w] = t;
    }
  }
}

// fitem: (segment, first chunk sum, chunk count, 0); one wave each
template <int MODE>
__global__ __launch_bounds__(kSegBlock) void k_seg1_fin(const int4* __restrict__ fitem, int nf,
                                                        const double* __restrict__ cpart, Epi e,
                                                        const int* done) {
  if (is_done(done)) return;
  const int wv = (int)blockIdx.x * (kSegBlock / 64) + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wv >= nf) return;
  const int4 it = fitem[wv];
  double t = 0.0;
  for (int k = lane; k < it.z; k += 64) t += cpart[it.y + k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if (lane == 0) {
    double dot = 0.0;
    seg_finish<MODE>(it.x, t, e, dot);
  }
}

// The coarse GEMV y = A c of the V(1,1) cycle with the restriction's
// finishing step folded in: every block copies c (n <= kGemvFinMax) into LDS
// and forms the long clusters' entries itself from their chunk sums, in the
// order and with the scaling of k_seg1_fin (so y is bitwise the same), then
// one wave per row as in k_gemv.
constexpr int kGemvFinMax = 4096;
constexpr int kGemvFinBlock = 256;
__global__ __launch_bounds__(kGemvFinBlock) void k_gemv_fin(int n, const double* __restrict__ A,
                                                     const double* __restrict__ c,
                                                     const int4* __restrict__ fitem, int nf,
                                                     const double* __restrict__ cpart,
                                                     const double* __restrict__ scale, double* __restrict__ y,
                                                     const int* done) {
  if (is_done(done)) return;
  __shared__ double xs[kGemvFinMax];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < n; i += kGemvFinBlock) xs[i] = c[i];
  __syncthreads();
  for (int f = wv; f < nf; f += kGemvFinBlock / 64) {
    const int4 it = fitem[f];
    double t = 0.0;
    for (int k = lane; k < it.z; k += 64) t += cpart[it.y + k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) xs[it.x] = scale ? t * scale[it.x] : t;
  }
  __syncthreads();
  const int row = blockIdx.x * (kGemvFinBlock / 64) + wv;
  if (row >= n) return;
  const double* a = A + (size_t)row * n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = lane; c0 < n; c0 += 1024) {
    double av[16], xv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int q = c0 + 64 * k;
      av[k] = q < n ? a[q] : 0.0;
      xv[k] = q < n ? xs[q] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k & 3] += av[k] * xv[k];
  }
  double t = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if (lane == 0) y[row] = t;
}

bool restrict_gemv_fusable(const MergePlan& mp, int n) { return mp.nwitem > 0 && n > 0 && n <= kGemvFinMax; }

void launch_restrict_gemv(const MergePlan& mp, const double* v_sorted, const double* val, const double* scale,
                          double* c, int n, const double* Ainv, double* yc, const int* done, hipStream_t s) {
  Epi e{};
  e.out = c;
  e.scale = scale;
  const int grid = cdiv(mp.nwitem, kSegBlock / 64);
  if (val) {
    if (scale)
      k_seg1<EPI_SCALE, true, false><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, nullptr, val, v_sorted, e,
                                                               mp.cpart, done);
    else
      k_seg1<EPI_STORE, true, false><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, nullptr, val, v_sorted, e,
                                                               mp.cpart, done);
  } else {
    if (scale)
      k_seg1<EPI_SCALE, false, false><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, nullptr, nullptr, v_sorted,
                                                                e, mp.cpart, done);
    else
      k_seg1<EPI_STORE, false, false><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, nullptr, nullptr, v_sorted,
                                                                e, mp.cpart, done);
  }
  k_gemv_fin<<<cdiv(n, kGemvFinBlock / 64), kGemvFinBlock, 0, s>>>(n, Ainv, c, mp.fitem, mp.nfitem, mp.cpart, scale, yc, done);
}

void launch_restrict_gemv_xp(const MergePlan& mp, const int* perm, const double* r, const double* e1, double lam,
                             const double* scale, const SellPlan& xp, const double* xpart, double* c, int n,
                             const double* Ainv, double* yc, const int* done, hipStream_t s) {
  Epi e{};
  e.out = c;
  e.scale = scale;
  e.r = r;
  e.p = e1;
  e.lam = lam;
  e.xbase = xp.sbase;
  e.xpos = xp.pos;
  e.xpart = xpart;
  const int grid = cdiv(mp.nwitem, kSegBlock / 64);
  k_seg1<EPI_SCALE, false, true, true><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, perm, nullptr, nullptr, e,
                                                                  mp.cpart, done);
  k_gemv_fin<<<cdiv(n, kGemvFinBlock / 64), kGemvFinBlock, 0, s>>>(n, Ainv, c, mp.fitem, mp.nfitem, mp.cpart, scale, yc, done);
}

template <int MODE>
static void seg1_mode(const MergePlan& mp, const int* idx, const double* val, const double* v,
                      const Epi& e, const int* done, hipStream_t s) {
  const int grid = cdiv(mp.nwitem, kSegBlock / 64);
  if (val && idx)
    k_seg1<MODE, true, true><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, idx, val, v, e, mp.cpart, done);
  else if (idx)
    k_seg1<MODE, false, true><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, idx, nullptr, v, e, mp.cpart,
                                                         done);
  else if (val)
    k_seg1<MODE, true, false><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, nullptr, val, v, e, mp.cpart,
                                                         done);
  else
    k_seg1<MODE, false, false><<<grid, kSegBlock, 0, s>>>(mp.witem, mp.nwitem, nullptr, nullptr, v, e,
                                                          mp.cpart, done);
  if (mp.nfitem > 0)
    k_seg1_fin<MODE><<<cdiv(mp.nfitem, kSegBlock / 64), kSegBlock, 0, s>>>(mp.fitem, mp.nfitem, mp.cpart, e,
                                                                           done);
}

// Collapse n block partials into partials[0] (one block, fixed order).
__global__ __launch_bounds__(kBlock) void k_collapse(double* partials, int n, const int* done) {
  if (is_done(done)) return;
  __shared__ double red[kBlock / 64];
  const double t = sum_parts<kBlock>(partials, n, red);
  if (threadIdx.x == 0) partials[0] = t;
}

template <int MODE>
static int segsum_mode(const MergePlan& mp, const int* seg_end, const int* idx,
                       const double* val, const double* v, const Epi& e, const int* done,
                       hipStream_t s) {
  const int nfix = std::max(1, cdiv(mp.nspan, kBlock / 64));
  const int nslots = mp.nblocks + nfix;
  if (val)
    k_segsum<MODE, false><<<mp.nblocks, kBlock, 0, s>>>(seg_end, idx, val, v, mp.coord, mp.head,
                                                       mp.tail, mp.nseg, nslots, e, done);
  else
    k_segsum<MODE, true><<<mp.nblocks, kBlock, 0, s>>>(seg_end, idx, nullptr, v, mp.coord,
                                                      mp.head, mp.tail, mp.nseg, nslots, e,
                                                      done);
  if (mp.nspan > 0 || has_dot<MODE>())
    k_segfix<MODE><<<nfix, kBlock, 0, s>>>(mp.span, mp.nspan, mp.head, mp.tail, mp.nblocks, e,
                                           done);
  if (!has_dot<MODE>()) return 0;
  return collapse_parts(e.partials, nslots, done, s);
}

int collapse_parts(double* partials, int n, const int* done, hipStream_t s) {
  if (n <= kMaxParts) return n;
  k_collapse<<<1, kBlock, 0, s>>>(partials, n, done);
  return 1;
}

int launch_csc(const Sparse& X, const double* u, int mode, const Epi& e, const int* done,
               hipStream_t s, hipEvent_t mid) {
  if (X.sliced) return launch_sell(X.sell_csc, u, mode, e, done, s, nullptr, mid);
  const int n = launch_segsum(X.csc_plan, X.col_ptr + 1, X.row_idx, X.cval, u, mode, e, done, s);
  if (mid) (void)hipEventRecord(mid, s);
  return n;
}

int launch_segsum(const MergePlan& mp, const int* seg_end, const int* idx, const double* val,
                  const double* v, int mode, const Epi& e, const int* done, hipStream_t s) {
  if (mp.nwitem > 0) {
    switch (mode) {
      case EPI_STORE: seg1_mode<EPI_STORE>(mp, idx, val, v, e, done, s); return 0;
      case EPI_SCALE: seg1_mode<EPI_SCALE>(mp, idx, val, v, e, done, s); return 0;
      default: break;
    }
  }
  if (!idx) return 0;   // segment-ordered input: only the one-kernel form reads it
  if (mp.nblocks == 0) return 0;
  switch (mode) {
    case EPI_STORE: return segsum_mode<EPI_STORE>(mp, seg_end, idx, val, v, e, done, s);
    case EPI_APPLY: return segsum_mode<EPI_APPLY>(mp, seg_end, idx, val, v, e, done, s);
    case EPI_APPLY_DOT: return segsum_mode<EPI_APPLY_DOT>(mp, seg_end, idx, val, v, e, done, s);
    case EPI_RESID: return segsum_mode<EPI_RESID>(mp, seg_end, idx, val, v, e, done, s);
    case EPI_POST: return segsum_mode<EPI_POST>(mp, seg_end, idx, val, v, e, done, s);
    case EPI_TRUE: return segsum_mode<EPI_TRUE>(mp, seg_end, idx, val, v, e, done, s);
    case EPI_SCALE: return segsum_mode<EPI_SCALE>(mp, seg_end, idx, val, v, e, done, s);
  }
  return 0;
}


// ---------------------------------------------------------------------------
// Plan construction (setup only)
// ---------------------------------------------------------------------------
__global__ void k_block_seg_start(const int2* coord, const int* seg_ptr, int nblocks,
                                  int* out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nblocks) out[b] = seg_ptr[coord[b].x];
}

void free_merge_plan(MergePlan& mp) {
  if (mp.coord) (void)dev_free(mp.coord);
  if (mp.span) (void)dev_free(mp.span);
  if (mp.head) (void)dev_free(mp.head);
  if (mp.tail) (void)dev_free(mp.tail);
  if (mp.witem) (void)dev_free(mp.witem);
  if (mp.fitem) (void)dev_free(mp.fitem);
  if (mp.cpart) (void)dev_free(mp.cpart);
  mp = MergePlan{};
}

// The wave-item form of a plan whose segments are seg_ptr[0..nseg] (setup
// only): a wave per segment of up to kWaveSeg entries, longer ones in about
// equal chunks of at most kWaveSeg entries plus a finishing wave.
rr_status build_chunk_plan(MergePlan& mp, const int* d_seg_ptr, int nseg, hipStream_t s) {
  std::vector<int> ptr(nseg + 1);
  RR_HIP(hipMemcpyAsync(ptr.data(), d_seg_ptr, sizeof(int) * (nseg + 1), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  std::vector<int4> wi, fi;
  int np = 0;
  for (int q = 0; q < nseg; ++q) {
    const int a = ptr[q], z = ptr[q + 1];
    if (z < a) return fail(RR_ERR_DEVICE, "internal: decreasing segment offsets");
    if (z - a <= kWaveSeg) {
      wi.push_back(make_int4(q, a, z, -1));
      continue;
    }
    const int nc = cdiv(z - a, kWaveSeg);
    fi.push_back(make_int4(q, np, nc, 0));
    for (int c = 0; c < nc; ++c) {
      const int c0 = a + (int)((long long)(z - a) * c / nc), c1 = a + (int)((long long)(z - a) * (c + 1) / nc);
      wi.push_back(make_int4(q, c0, c1, np++));
    }
  }
  for (const int4& w : wi)
    if (w.z - w.y > kWaveSeg || w.w >= np) return fail(RR_ERR_DEVICE, "internal: segment item out of range");
  mp.nwitem = (int)wi.size();
  mp.nfitem = (int)fi.size();
  mp.ncpart = np;
  if (mp.nwitem) {
    RR_HIP(dmalloc(&mp.witem, sizeof(int4) * mp.nwitem));
    RR_HIP(hipMemcpyAsync(mp.witem, wi.data(), sizeof(int4) * mp.nwitem, hipMemcpyHostToDevice, s));
  }
  if (mp.nfitem) {
    RR_HIP(dmalloc(&mp.fitem, sizeof(int4) * mp.nfitem));
    RR_HIP(hipMemcpyAsync(mp.fitem, fi.data(), sizeof(int4) * mp.nfitem, hipMemcpyHostToDevice, s));
  }
  if (np) RR_HIP(dmalloc(&mp.cpart, sizeof(double) * np));
  RR_HIP(hipStreamSynchronize(s));
  return RR_OK;
}

rr_status build_xp_restrict(MergePlan& mp, const SellPlan& xp, const int* d_coff, int FC, int F, hipStream_t s) {
  free_merge_plan(mp);
  std::vector<int> ptr(FC + 1), sb(FC + 1);
  RR_HIP(hipMemcpyAsync(ptr.data(), d_coff, sizeof(int) * (FC + 1), hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(sb.data(), xp.sbase, sizeof(int) * (FC + 1), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  if (xp.S != FC || ptr[0] != 0 || ptr[FC] != F || sb[0] != 0 || sb[FC] != xp.nitems)
    return fail(RR_ERR_DEVICE, "internal: X P plan does not match the clusters");
  std::vector<int4> wi, fi;
  int np = 0;
  for (int q = 0; q < FC; ++q) {
    const int a = ptr[q], z = ptr[q + 1], p0 = sb[q], p1 = sb[q + 1];
    if (z < a || p1 < p0) return fail(RR_ERR_DEVICE, "internal: decreasing segment offsets");
    if (z - a <= kWaveSeg && p1 - p0 <= kXpPieces) {
      wi.push_back(make_int4(q, a, z, -1));
      continue;
    }
    const int nc = std::max(1, cdiv(z - a, kWaveSeg)), npc = cdiv(p1 - p0, kXpPieceItem);
    fi.push_back(make_int4(q, np, nc + npc, 0));
    for (int c = 0; c < nc; ++c) {
      const int c0 = a + (int)((long long)(z - a) * c / nc), c1 = a + (int)((long long)(z - a) * (c + 1) / nc);
      wi.push_back(make_int4(q, c0, c1, np++));
    }
    for (int c = 0; c < npc; ++c)
      wi.push_back(make_int4(-1 - q, p0 + c * kXpPieceItem, std::min(p1, p0 + (c + 1) * kXpPieceItem), np++));
  }
  for (const int4& w : wi) {
    const bool piece = w.x < 0;
    const int lim = piece ? xp.nitems : F, len = piece ? kXpPieceItem : kWaveSeg;
    if (w.y < 0 || w.z > lim || w.z - w.y > len || w.z < w.y || w.w >= np || (piece && w.w < 0))
      return fail(RR_ERR_DEVICE, "internal: segment item out of range");
  }
  mp.nseg = FC;
  mp.nwitem = (int)wi.size();
  mp.nfitem = (int)fi.size();
  mp.ncpart = np;
  RR_HIP(dmalloc(&mp.witem, sizeof(int4) * std::max<size_t>(1, wi.size())));
  if (!wi.empty()) RR_HIP(hipMemcpyAsync(mp.witem, wi.data(), sizeof(int4) * wi.size(), hipMemcpyHostToDevice, s));
  if (mp.nfitem) {
    RR_HIP(dmalloc(&mp.fitem, sizeof(int4) * mp.nfitem));
    RR_HIP(hipMemcpyAsync(mp.fitem, fi.data(), sizeof(int4) * mp.nfitem, hipMemcpyHostToDevice, s));
  }
  if (np) RR_HIP(dmalloc(&mp.cpart, sizeof(double) * np));
  RR_HIP(hipStreamSynchronize(s));
  return RR_OK;
}

// seg_end = ptr + 1 (nseg entries), seg_ptr = ptr (nseg + 1 entries).
rr_status build_merge_plan(MergePlan& mp, const int* d_seg_end, const int* d_seg_ptr, int nseg,
                           int nnz, hipStream_t s) {
  free_merge_plan(mp);
  mp.nseg = nseg;
  mp.nnz = nnz;
  const long long total = (long long)nseg + nnz;
  if (total == 0) return RR_OK;
  if (total >= INT_MAX) return fail(RR_ERR_INVALID_ARG, "merge plan: segments + nonzeros >= 2^31");
  mp.nblocks = cdiv(total, kMergeTile);
  RR_HIP(dmalloc(&mp.coord, sizeof(int2) * (mp.nblocks + 1)));
  RR_HIP(dmalloc(&mp.head, sizeof(double) * mp.nblocks));
  RR_HIP(dmalloc(&mp.tail, sizeof(double) * mp.nblocks));
  k_merge_coord<<<cdiv(mp.nblocks + 1, kBlock), kBlock, 0, s>>>(d_seg_end, nseg, nnz, mp.nblocks,
                                                               mp.coord);
  int* d_start = nullptr;
  RR_HIP(dmalloc(&d_start, sizeof(int) * mp.nblocks));
  k_block_seg_start<<<cdiv(mp.nblocks, kBlock), kBlock, 0, s>>>(mp.coord, d_seg_ptr, mp.nblocks,
                                                               d_start);
  std::vector<int2> coord(mp.nblocks + 1);
  std::vector<int> start(mp.nblocks);
  RR_HIP(hipMemcpyAsync(coord.data(), mp.coord, sizeof(int2) * (mp.nblocks + 1),
                        hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(start.data(), d_start, sizeof(int) * mp.nblocks, hipMemcpyDeviceToHost,
                        s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(d_start));
  // Segments that cross tiles: a run of tiles b_a..b_z that all begin inside
  // segment s; s started in tile b_a - 1 and ends in tile b_z.
  std::vector<int4> spans;
  int b = 1;
  while (b < mp.nblocks) {
    const bool mid = start[b] < coord[b].y;
    if (!mid) {
      ++b;
      continue;
    }
    const int seg = coord[b].x;
    int bz = b;
    while (bz + 1 < mp.nblocks && coord[bz + 1].x == seg && start[bz + 1] < coord[bz + 1].y) ++bz;
    spans.push_back(make_int4(seg, b - 1, bz, 0));
    b = bz + 1;
  }
  mp.nspan = (int)spans.size();
  if (mp.nspan) {
    RR_HIP(dmalloc(&mp.span, sizeof(int4) * mp.nspan));
    RR_HIP(hipMemcpyAsync(mp.span, spans.data(), sizeof(int4) * mp.nspan, hipMemcpyHostToDevice,
                          s));
    RR_HIP(hipStreamSynchronize(s));
  }
  return RR_OK;
}

// ---------------------------------------------------------------------------
// Input validation and the CSC transpose (setup only)
// ---------------------------------------------------------------------------
__global__ void k_validate(const int* ptr, const int* idx, const double* val, int N, int F,
                           int nnz, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > N) return;
  if (i == 0 && ptr[0] != 0) atomicOr(flag, 1);
  if (i == N) {
    if (ptr[N] != nnz) atomicOr(flag, 1);
    return;
  }
  const int a = ptr[i], b = ptr[i + 1];
  if (b < a || a < 0 || b > nnz) {
    atomicOr(flag, 1);
    return;
  }
  int prev = -1;
  for (int e = a; e < b; ++e) {
    const int c = idx[e];
    if (c < 0 || c >= F) atomicOr(flag, 2);
    if (c <= prev) atomicOr(flag, 4);
    prev = c;
    if (val) {
      const double x = val[e];
      if (!(x == x) || x == __builtin_inf() || x == -__builtin_inf()) atomicOr(flag, 8);
      if (x < 0.0) atomicOr(flag, 16);
    }
  }
}

rr_status validate_csr(const Sparse& X, hipStream_t s) {
  int* d_flag = nullptr;
  RR_HIP(dmalloc(&d_flag, sizeof(int)));
  RR_HIP(hipMemsetAsync(d_flag, 0, sizeof(int), s));
  k_validate<<<cdiv(X.N + 1, kBlock), kBlock, 0, s>>>(X.row_ptr, X.col_idx, X.val, X.N, X.F,
                                                      X.nnz, d_flag);
  int flag = 0;
  RR_HIP(hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(d_flag));
  if (flag & 1) return fail(RR_ERR_INVALID_ARG, "X: row_ptr is not a valid CSR pointer array");
  if (flag & 2) return fail(RR_ERR_INVALID_ARG, "X: column index out of range");
  if (flag & 4) return fail(RR_ERR_INVALID_ARG, "X: column indices not strictly increasing in a row");
  if (flag & 8) return fail(RR_ERR_INVALID_ARG, "X: non-finite value");
  return (flag & 16) ? RR_ERR_UNSUPPORTED : RR_OK;   // caller records "has negatives"
}

__global__ void k_expand_rows(const int* ptr, int N, int* row_of) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) row_of[e] = i;
}

__global__ void k_iota(int* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

__global__ void k_lower_bound_ptr(const int* keys, int n, int nseg, int* ptr) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nseg) return;
  int lo = 0, hi = n;
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (keys[m] < j)
      lo = m + 1;
    else
      hi = m;
  }
  ptr[j] = lo;
}

__global__ void k_gather_csc(const int* order, const int* row_of, const double* val, int nnz,
                             int* row_idx, double* cval) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int e = order[k];
  row_idx[k] = row_of[e];
  if (val) cval[k] = val[e];
}

static unsigned bits_for(int n) {
  unsigned b = 1;
  while ((1ll << b) < (long long)n) ++b;
  return b;
}

// ---------------------------------------------------------------------------
// Feature renumbering (setup only): internal feature order = descending
// column count, ties in the caller's order, so the most popular columns'
// entries of every F-vector share cache lines and the CSR gathers of v hit
// the L1.  fperm[new] = caller index, finv[caller] = new index.
// ---------------------------------------------------------------------------
__global__ void k_col_count(const int* col_idx, int nnz, int* cnt) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x)
    atomicAdd(&cnt[col_idx[e]], 1);
}

__global__ void k_invert(const int* fperm, int F, int* finv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < F) finv[fperm[i]] = i;
}

// key = row << 32 | new column, so a radix sort orders each row by new index
__global__ void k_row_keys(const int* ptr, const int* col_idx, const int* finv, int N,
                           unsigned long long* keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int e = ptr[i]; e < ptr[i + 1]; ++e)
    keys[e] = ((unsigned long long)i << 32) | (unsigned)finv[col_idx[e]];
}

__global__ void k_keys_to_cols(const unsigned long long* keys, int nnz, int* col_idx) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) col_idx[e] = (int)(keys[e] & 0xffffffffull);
}

rr_status renumber_features(Sparse& X, int* fperm, int* finv, hipStream_t s) {
  const int F = X.F, nnz = X.nnz, N = X.N;
  int *cnt = nullptr, *cnt_out = nullptr, *iota = nullptr;
  RR_HIP(dmalloc(&cnt, sizeof(int) * F));
  RR_HIP(dmalloc(&cnt_out, sizeof(int) * F));
  RR_HIP(dmalloc(&iota, sizeof(int) * F));
  RR_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * F, s));
  if (nnz) k_col_count<<<std::min(4096, cdiv(nnz, kBlock)), kBlock, 0, s>>>(X.col_idx, nnz, cnt);
  k_iota<<<cdiv(F, kBlock), kBlock, 0, s>>>(iota, F);
  size_t tmp_bytes = 0;
  RR_HIP(rocprim::radix_sort_pairs_desc(nullptr, tmp_bytes, cnt, cnt_out, iota, fperm, (size_t)F, 0u,
                                        32u, s));
  void* tmp = nullptr;
  RR_HIP(dmalloc(&tmp, std::max<size_t>(tmp_bytes, 1)));
  RR_HIP(rocprim::radix_sort_pairs_desc(tmp, tmp_bytes, cnt, cnt_out, iota, fperm, (size_t)F, 0u, 32u,
                                        s));
  k_invert<<<cdiv(F, kBlock), kBlock, 0, s>>>(fperm, F, finv);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(tmp));
  RR_HIP(dev_free(cnt));
  RR_HIP(dev_free(cnt_out));
  RR_HIP(dev_free(iota));
  if (nnz == 0) return RR_OK;
  unsigned long long *keys = nullptr, *keys_out = nullptr;
  RR_HIP(dmalloc(&keys, sizeof(unsigned long long) * nnz));
  RR_HIP(dmalloc(&keys_out, sizeof(unsigned long long) * nnz));
  k_row_keys<<<cdiv(N, kBlock), kBlock, 0, s>>>(X.row_ptr, X.col_idx, finv, N, keys);
  unsigned end_bit = 32 + bits_for(N);
  tmp_bytes = 0;
  if (X.binary) {
    RR_HIP(rocprim::radix_sort_keys(nullptr, tmp_bytes, keys, keys_out, (size_t)nnz, 0u, end_bit, s));
    RR_HIP(dmalloc(&tmp, std::max<size_t>(tmp_bytes, 1)));
    RR_HIP(rocprim::radix_sort_keys(tmp, tmp_bytes, keys, keys_out, (size_t)nnz, 0u, end_bit, s));
  } else {
    double* vout = nullptr;
    RR_HIP(dmalloc(&vout, sizeof(double) * nnz));
    RR_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys, keys_out, X.val, vout, (size_t)nnz, 0u,
                                     end_bit, s));
    RR_HIP(dmalloc(&tmp, std::max<size_t>(tmp_bytes, 1)));
    RR_HIP(rocprim::radix_sort_pairs(tmp, tmp_bytes, keys, keys_out, X.val, vout, (size_t)nnz, 0u,
                                     end_bit, s));
    RR_HIP(hipMemcpyAsync(X.val, vout, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    RR_HIP(hipStreamSynchronize(s));
    RR_HIP(dev_free(vout));
  }
  k_keys_to_cols<<<cdiv(nnz, kBlock), kBlock, 0, s>>>(keys_out, nnz, X.col_idx);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(tmp));
  RR_HIP(dev_free(keys));
  RR_HIP(dev_free(keys_out));
  return RR_OK;
}

// CSC by a stable radix sort of (column, CSR position): rows stay increasing
// inside every column, so the transpose is deterministic.
rr_status build_csc(Sparse& X, hipStream_t s) {
  const int nnz = X.nnz;
  RR_HIP(dmalloc(&X.col_ptr, sizeof(int) * (X.F + 1)));
  RR_HIP(dmalloc(&X.row_idx, sizeof(int) * std::max(nnz, 1)));
  if (!X.binary) RR_HIP(dmalloc(&X.cval, sizeof(double) * std::max(nnz, 1)));
  if (nnz == 0) {
    RR_HIP(hipMemsetAsync(X.col_ptr, 0, sizeof(int) * (X.F + 1), s));
    return RR_OK;
  }
  int *row_of = nullptr, *pos = nullptr, *keys_out = nullptr, *pos_out = nullptr;
  RR_HIP(dmalloc(&row_of, sizeof(int) * nnz));
  RR_HIP(dmalloc(&pos, sizeof(int) * nnz));
  RR_HIP(dmalloc(&keys_out, sizeof(int) * nnz));
  RR_HIP(dmalloc(&pos_out, sizeof(int) * nnz));
  k_expand_rows<<<cdiv(X.N, kBlock), kBlock, 0, s>>>(X.row_ptr, X.N, row_of);
  k_iota<<<cdiv(nnz, kBlock), kBlock, 0, s>>>(pos, nnz);
  size_t tmp_bytes = 0;
  const unsigned end_bit = bits_for(X.F);
  RR_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, X.col_idx, keys_out, pos, pos_out,
                                   (size_t)nnz, 0u, end_bit, s));
  void* tmp = nullptr;
  RR_HIP(dmalloc(&tmp, std::max<size_t>(tmp_bytes, 1)));
  RR_HIP(rocprim::radix_sort_pairs(tmp, tmp_bytes, X.col_idx, keys_out, pos, pos_out, (size_t)nnz,
                                   0u, end_bit, s));
  k_lower_bound_ptr<<<cdiv(X.F + 1, kBlock), kBlock, 0, s>>>(keys_out, nnz, X.F, X.col_ptr);
  k_gather_csc<<<cdiv(nnz, kBlock), kBlock, 0, s>>>(pos_out, row_of, X.binary ? nullptr : X.val,
                                                    nnz, X.row_idx, X.cval);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(dev_free(tmp));
  RR_HIP(dev_free(row_of));
  RR_HIP(dev_free(pos));
  RR_HIP(dev_free(keys_out));
  RR_HIP(dev_free(pos_out));
  if (X.binary) return RR_OK;   // 0/1 matrices use the sliced-ELL plans
  return build_merge_plan(X.csc_plan, X.col_ptr + 1, X.col_ptr, X.F, nnz, s);
}

}  // namespace rr
