// Sliced-ELL segmented gather-sums with the gathered vector in LDS: the
// operator's two sparse passes for 0/1 matrices.
//
// A pass computes out_s = sum_{e in segment s} v[g_e] for segments s (rows of
// X for u = X v, columns of X for t = X^T u).  The gathered index range is cut
// into slices of W entries whose part of v fits in LDS (W = 16384 FP64 =
// 128 KB, plus one zero entry used for padding).  Every nonempty (segment,
// slice) pair gets one output slot; slots of a segment are consecutive, in
// slice order.  Pairs of one slice are processed by workgroups that first
// copy the slice's part of v into LDS:
//   * pairs with at most 512 entries are sorted by length and packed 64 to a
//     wave task, lane l summing pair l; entry k of lane l is stored at
//     base + 64 k + l (uint16, local index), padded with the zero entry to
//     the task's longest pair, so every load instruction reads 128
//     consecutive bytes;
//   * longer pairs are one wave task each, stored contiguously and padded to
//     a multiple of 512 entries; lane l reads 8 entries (16 bytes) per 512,
//     then the wave adds its lanes in a fixed butterfly.
// A reduction kernel then adds each segment's slots in slice order and
// applies the epilogue.  Each sum's order is fixed by the plan, so results
// are bitwise reproducible.
#include <algorithm>
#include <numeric>

#include "rr_device.h"

namespace rr {

constexpr int kHeavyLen = 512;      // pairs longer than this get a whole wave
constexpr int kLaneUnroll = 32;     // index loads in flight per lane (lane tasks)
constexpr int kWaveUnroll = 16;     // 16-byte loads in flight per lane (wave tasks)

template <int NTHREADS, int MAXN>
__device__ inline void fill_slice(double* dst, const double* __restrict__ src, int n) {
  constexpr int PER = (MAXN + NTHREADS - 1) / NTHREADS;
  double t[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * NTHREADS;
    t[k] = (i < n) ? src[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * NTHREADS;
    if (i < MAXN) dst[i] = t[k];
  }
}

// task.x: kind (0 lane task, 1 wave task); task.y: offset of its indices
// (uint16 units for lane tasks, 16-byte units for wave tasks); task.z: length
// (longest pair for lane tasks, 512-entry groups for wave tasks); task.w:
// first lane-slot entry (lane tasks) or the output slot (wave tasks).
__global__ __launch_bounds__(kSliceBlock) void k_sell(const int4* __restrict__ blk,
                                                     const int4* __restrict__ task,
                                                     const uint16_t* __restrict__ idx,
                                                     const int* __restrict__ lane_slot,
                                                     const double* __restrict__ v, int gdim,
                                                     int W, double* __restrict__ out,
                                                     const int* done, StageArgs stage) {
  if (is_done(done)) return;
  if (stage.sc) {   // convergence check of the preceding x/r update
    __shared__ double red_s[kSliceWaves];
    double rz_unused;
    if (stage_update<kSliceBlock>(stage, red_s, rz_unused)) return;
  }
  __shared__ double vs[kSliceRows + 1];
  const int4 b = blk[blockIdx.x];
  const int r = b.x;
  const int g0 = r * W;
  fill_slice<kSliceBlock, kSliceRows + 1>(vs, v + g0, min(W, gdim - g0));
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = b.y + w; t < b.z; t += kSliceWaves) {
    const int4 tk = task[t];
    if (tk.x == 0) {
      const uint16_t* p = idx + tk.y + lane;
      const int m = tk.z;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int k = 0;
      for (; k + kLaneUnroll <= m; k += kLaneUnroll) {
        uint16_t q[kLaneUnroll];
#pragma unroll
        for (int j = 0; j < kLaneUnroll; ++j) q[j] = p[(size_t)(k + j) * 64];
#pragma unroll
        for (int j = 0; j < kLaneUnroll; ++j) acc[j & 3] += vs[q[j]];
      }
      if (k < m) {   // the rest, loads issued together
        uint16_t q[kLaneUnroll];
#pragma unroll
        for (int j = 0; j < kLaneUnroll; ++j) q[j] = (k + j < m) ? p[(size_t)(k + j) * 64] : (uint16_t)0;
#pragma unroll
        for (int j = 0; j < kLaneUnroll; ++j)
          if (k + j < m) acc[j & 3] += vs[q[j]];
      }
      const double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
      const int slot = lane_slot[tk.w + lane];
      if (slot >= 0) out[slot] = s;
    } else {
      const uint4* p = reinterpret_cast<const uint4*>(idx) + tk.y + lane;
      const int ng = tk.z;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int g = 0;
      for (; g + kWaveUnroll <= ng; g += kWaveUnroll) {
        uint4 q[kWaveUnroll];
#pragma unroll
        for (int j = 0; j < kWaveUnroll; ++j) q[j] = p[(size_t)(g + j) * 64];
#pragma unroll
        for (int j = 0; j < kWaveUnroll; ++j) {
          const unsigned wds[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            acc[(2 * h) & 3] += vs[wds[h] & 0xffffu];
            acc[(2 * h + 1) & 3] += vs[wds[h] >> 16];
          }
        }
      }
      if (g < ng) {   // the rest, loads issued together
        uint4 q[kWaveUnroll];
#pragma unroll
        for (int j = 0; j < kWaveUnroll; ++j)
          q[j] = (g + j < ng) ? p[(size_t)(g + j) * 64] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < kWaveUnroll; ++j) {
          if (g + j < ng) {
            const unsigned wds[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              acc[(2 * h) & 3] += vs[wds[h] & 0xffffu];
              acc[(2 * h + 1) & 3] += vs[wds[h] >> 16];
            }
          }
        }
      }
      double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) out[tk.w] = s;
    }
  }
}

// segment s: t = sum of its slots in slice order, then the epilogue
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_sell_reduce(const double* __restrict__ slots,
                                                       const int* __restrict__ sbase, int S,
                                                       Epi e, const int* done) {
  if (is_done(done)) return;
  double dot = 0.0;
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += gridDim.x * kBlock) {
    const int a = sbase[s], z = sbase[s + 1];
    double t = 0.0;
    for (int k0 = a; k0 < z; k0 += 8) {
      double pv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) pv[j] = (k0 + j < z) ? slots[k0 + j] : 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (k0 + j < z) t += pv[j];
    }
    seg_finish<MODE>(s, t, e, dot);
  }
  if constexpr (has_dot<MODE>()) store_block_partial<kBlock>(dot, e.partials, blockIdx.x);
}

int sell_reduce_grid(int S) { return std::max(1, std::min(256, cdiv(S, kBlock))); }

template <int MODE>
static void sell_reduce_mode(const SellPlan& sp, const Epi& e, const int* done, hipStream_t s) {
  k_sell_reduce<MODE><<<sell_reduce_grid(sp.S), kBlock, 0, s>>>(sp.slots, sp.sbase, sp.S, e, done);
}

int launch_sell(const SellPlan& sp, const double* v, int mode, const Epi& e, const int* done,
                hipStream_t s, const StageArgs* stage) {
  StageArgs st{};
  if (stage) st = *stage;
  if (sp.nblk > 0)
    k_sell<<<sp.nblk, kSliceBlock, 0, s>>>(sp.blk, sp.task, sp.idx, sp.lane_slot, v, sp.gdim,
                                          sp.W, sp.slots, done, st);
  else if (stage)
    launch_stage_update(*stage, s);
  switch (mode) {
    case EPI_STORE: sell_reduce_mode<EPI_STORE>(sp, e, done, s); break;
    case EPI_APPLY: sell_reduce_mode<EPI_APPLY>(sp, e, done, s); break;
    case EPI_APPLY_DOT: sell_reduce_mode<EPI_APPLY_DOT>(sp, e, done, s); break;
    case EPI_RESID: sell_reduce_mode<EPI_RESID>(sp, e, done, s); break;
    case EPI_POST: sell_reduce_mode<EPI_POST>(sp, e, done, s); break;
    case EPI_TRUE: sell_reduce_mode<EPI_TRUE>(sp, e, done, s); break;
    case EPI_SCALE: sell_reduce_mode<EPI_SCALE>(sp, e, done, s); break;
  }
  return sell_reduce_grid(sp.S);
}

void free_sell(SellPlan& sp) {
  if (sp.idx) (void)hipFree(sp.idx);
  if (sp.task) (void)hipFree(sp.task);
  if (sp.blk) (void)hipFree(sp.blk);
  if (sp.lane_slot) (void)hipFree(sp.lane_slot);
  if (sp.sbase) (void)hipFree(sp.sbase);
  if (sp.slots) (void)hipFree(sp.slots);
  sp = SellPlan{};
}

// Host-side construction from a segment-major pattern (ptr[S+1], gidx sorted
// inside every segment).  Setup only.
rr_status build_sell(SellPlan& sp, const std::vector<int>& ptr, const std::vector<int>& gidx,
                     int S, int gdim, int num_cu, hipStream_t s) {
  free_sell(sp);
  const int W = kSliceRows;
  const int R = std::max(1, cdiv(gdim, W));
  sp.S = S;
  sp.gdim = gdim;
  sp.W = W;
  sp.R = R;
  // nonempty (segment, slice) pairs in (segment, slice) order = slot order
  struct Pair {
    int start, len;
  };
  std::vector<Pair> pairs;
  std::vector<int> pslice;
  std::vector<int> sbase(S + 1, 0);
  pairs.reserve(ptr[S] / 2 + S);
  for (int q = 0; q < S; ++q) {
    sbase[q] = (int)pairs.size();
    int e = ptr[q];
    const int z = ptr[q + 1];
    while (e < z) {
      const int r = gidx[e] / W;
      int f = e;
      while (f < z && gidx[f] / W == r) ++f;
      pairs.push_back({e, f - e});
      pslice.push_back(r);
      e = f;
    }
  }
  sbase[S] = (int)pairs.size();
  sp.nslots = (int)pairs.size();
  // per slice: heavy pairs (own wave) and light pairs (64 per wave, by length)
  std::vector<std::vector<int>> light(R), heavy(R);
  for (int i = 0; i < (int)pairs.size(); ++i)
    (pairs[i].len > kHeavyLen ? heavy : light)[pslice[i]].push_back(i);
  std::vector<uint16_t> idx;
  std::vector<int4> tasks;
  std::vector<int> lane_slot;
  std::vector<long long> tcost;
  std::vector<int> tslice;
  const uint16_t pad = (uint16_t)W;   // index of the zero entry
  for (int r = 0; r < R; ++r) {
    const int g0 = r * W;
    for (int i : heavy[r]) {
      while (idx.size() % 8) idx.push_back(pad);
      const int base16 = (int)(idx.size() / 8);
      const int len = pairs[i].len;
      const int ng = cdiv(len, 512);
      for (int k = 0; k < ng * 512; ++k)
        idx.push_back(k < len ? (uint16_t)(gidx[pairs[i].start + k] - g0) : pad);
      tasks.push_back(make_int4(1, base16, ng, i));
      tcost.push_back((long long)ng * 8 + 8);
      tslice.push_back(r);
    }
    std::vector<int>& lt = light[r];
    std::stable_sort(lt.begin(), lt.end(),
                     [&](int a, int b) { return pairs[a].len > pairs[b].len; });
    for (size_t c = 0; c < lt.size(); c += 64) {
      const int nv = (int)std::min<size_t>(64, lt.size() - c);
      const int m = pairs[lt[c]].len;
      const int base = (int)idx.size();
      idx.resize(idx.size() + (size_t)m * 64, pad);
      for (int l = 0; l < nv; ++l) {
        const Pair& pa = pairs[lt[c + l]];
        for (int k = 0; k < pa.len; ++k)
          idx[base + (size_t)k * 64 + l] = (uint16_t)(gidx[pa.start + k] - g0);
      }
      const int ls = (int)lane_slot.size();
      for (int l = 0; l < 64; ++l) lane_slot.push_back(l < nv ? lt[c + l] : -1);
      tasks.push_back(make_int4(0, base, m, ls));
      tcost.push_back((long long)m + 8);
      tslice.push_back(r);
    }
  }
  // workgroups: tasks of one slice, balanced on cost, about num_cu in total
  long long total = 0;
  for (long long c : tcost) total += c;
  std::vector<int4> blks;
  std::vector<int4> tasks_sorted;
  tasks_sorted.reserve(tasks.size());
  const long long per_blk = std::max(1LL, total / std::max(1, num_cu));
  size_t t = 0;
  while (t < tasks.size()) {
    const int r = tslice[t];
    size_t u = t;
    long long c = 0;
    while (u < tasks.size() && tslice[u] == r && (c < per_blk || u == t)) c += tcost[u++];
    // inside a workgroup, heaviest tasks first so the waves' round robin balances
    std::vector<size_t> ord(u - t);
    std::iota(ord.begin(), ord.end(), t);
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return tcost[a] > tcost[b]; });
    const int first = (int)tasks_sorted.size();
    for (size_t o : ord) tasks_sorted.push_back(tasks[o]);
    blks.push_back(make_int4(r, first, (int)tasks_sorted.size(), 0));
    t = u;
  }
  sp.nblk = (int)blks.size();
  sp.ntask = (int)tasks_sorted.size();
  while (idx.size() % 8) idx.push_back(pad);
  if (idx.empty()) idx.resize(8, pad);
  if (lane_slot.empty()) lane_slot.push_back(-1);
  RR_HIP(hipMalloc(&sp.idx, sizeof(uint16_t) * idx.size()));
  RR_HIP(hipMalloc(&sp.task, sizeof(int4) * std::max<size_t>(1, tasks_sorted.size())));
  RR_HIP(hipMalloc(&sp.blk, sizeof(int4) * std::max<size_t>(1, blks.size())));
  RR_HIP(hipMalloc(&sp.lane_slot, sizeof(int) * lane_slot.size()));
  RR_HIP(hipMalloc(&sp.sbase, sizeof(int) * sbase.size()));
  RR_HIP(hipMalloc(&sp.slots, sizeof(double) * std::max(1, sp.nslots)));
  RR_HIP(hipMemcpyAsync(sp.idx, idx.data(), sizeof(uint16_t) * idx.size(), hipMemcpyHostToDevice, s));
  if (!tasks_sorted.empty())
    RR_HIP(hipMemcpyAsync(sp.task, tasks_sorted.data(), sizeof(int4) * tasks_sorted.size(),
                          hipMemcpyHostToDevice, s));
  if (!blks.empty())
    RR_HIP(hipMemcpyAsync(sp.blk, blks.data(), sizeof(int4) * blks.size(), hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(sp.lane_slot, lane_slot.data(), sizeof(int) * lane_slot.size(),
                        hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(sp.sbase, sbase.data(), sizeof(int) * sbase.size(), hipMemcpyHostToDevice, s));
  RR_HIP(hipStreamSynchronize(s));
  sp.idx_bytes = (long long)idx.size() * 2;
  return RR_OK;
}

rr_status build_sell_plans(Sparse& X, hipStream_t s) {
  if (!X.binary) return RR_OK;   // valued matrices use the row-group / merge-path kernels
  std::vector<int> rp(X.N + 1), ci(std::max(X.nnz, 1)), cp(X.F + 1), ri(std::max(X.nnz, 1));
  RR_HIP(hipMemcpyAsync(rp.data(), X.row_ptr, sizeof(int) * (X.N + 1), hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(cp.data(), X.col_ptr, sizeof(int) * (X.F + 1), hipMemcpyDeviceToHost, s));
  if (X.nnz) {
    RR_HIP(hipMemcpyAsync(ci.data(), X.col_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToHost, s));
    RR_HIP(hipMemcpyAsync(ri.data(), X.row_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToHost, s));
  }
  RR_HIP(hipStreamSynchronize(s));
  RR_TRY(build_sell(X.sell_csr, rp, ci, X.N, X.F, X.num_cu, s));
  RR_TRY(build_sell(X.sell_csc, cp, ri, X.F, X.N, X.num_cu, s));
  return RR_OK;
}

}  // namespace rr
