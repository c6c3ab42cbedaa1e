// Sliced-ELL segmented gather-sums with the gathered vector in LDS: the
// operator's two sparse passes for 0/1 matrices.
//
// A pass computes out_s = sum_{e in segment s} v[g_e] for segments s (rows of
// X for u = X v, columns of X for t = X^T u).  The gathered index range is cut
// into slices of W entries whose part of v fits in LDS (W = 16384 FP64 =
// 128 KB, plus one zero entry used for padding).  Every nonempty (segment,
// slice) pair produces one partial sum, or one per piece when it is cut into
// pieces to keep lane streams short or a long pair's wave task near the
// others' load.  Workgroups own one slice each; they
// copy its part of v into LDS and then work through wave tasks:
//   * lane tasks: 64 lane streams of uint16 local indexes, entry k of lane l
//     stored at base + 256 (k / 4) + 4 l + k % 4, so a lane loads four
//     consecutive entries (8 bytes) at a time and every load instruction
//     reads 512 consecutive bytes.  A lane task is a stack of layers of 64
//     pairs of nearly equal length: lane l takes the l-th pair of every
//     layer, padded with the zero entry to the layer's longest; bit 15 marks
//     the layer's last entry in every lane, where all 64 lanes write their
//     running sums together (layer c to base + 64 c + l) and restart.  The
//     task is padded to a multiple of 4 entries;
//   * wave tasks: one long pair, stored contiguously and padded to a
//     multiple of 64 entries; lane l reads 8 entries (16 bytes) of every full
//     512 and one entry (2 bytes) of every 64 of the rest, then the wave adds
//     its lanes in a fixed butterfly.
// Tasks are spread over the waves of a slice's workgroups by cost, and every
// wave fetches its task descriptors in one load before the slice copy.  A
// reduction kernel then adds each segment's partial sums in slice order
// (reading them through a position index) and applies the epilogue.  Every
// sum's order is fixed by the plan, so results are bitwise reproducible.
#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <queue>

#include "rr_device.h"

namespace rr {

constexpr int kLaneGroup = 4;       // lane-task entries per load (8 bytes)
constexpr int kLaneUnroll = 8;      // loads (of kLaneGroup entries) in flight per lane
constexpr int kWaveUnroll = 16;     // 16-byte loads in flight per lane (wave tasks)
constexpr unsigned kEndFlag = 0x8000u;
constexpr unsigned kLocalMask = 0x7fffu;

// task.x: kind (0 lane task, 1 wave task); task.y: offset of its indexes
// (uint16 units for lane tasks, 16-byte units for wave tasks); task.z:
// length (longest lane stream; for wave tasks 16 x the 512-entry groups +
// the 64-entry tail groups); task.w: first output position.  Wave w of workgroup b runs tasks [wrange[17 b + w],
// wrange[17 b + w + 1]) of slice bslice[b].
// T is the type of the gathered vector, of the LDS slice and of the sums
// (double, or float for the single-precision inner solves).
template <typename T>
__device__ inline void sell_body(const int* __restrict__ wrange, const int* __restrict__ bslice,
                                 const int4* __restrict__ task, const uint16_t* __restrict__ idx,
                                 const T* __restrict__ v, int gdim, int W, T* __restrict__ out,
                                 const int* done, const StageArgs& stage) {
  if (is_done(done)) return;
  __shared__ __align__(16) T vs[kSliceRows + 1];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int t0 = wrange[blockIdx.x * (kSliceWaves + 1) + w];
  const int t1 = wrange[blockIdx.x * (kSliceWaves + 1) + w + 1];
  int4 my = make_int4(0, 0, 0, 0);
  if (t0 + lane < t1) my = task[t0 + lane];
  const int g0 = bslice[blockIdx.x] * W;
  fill_slice(vs, v + g0, min(W, gdim - g0));
  // Lane-task batches of kLaneUnroll 8-byte loads run one ahead: `pre` holds
  // the loads of the next batch (the rest of this task, else the first batch
  // of the next task if that is a lane task described by the same
  // descriptor load), issued before the current batch is summed.
  uint2 pre[kLaneUnroll];
  bool have = false;
  auto issue = [&](int base, int g, int ng) {
    const uint2* p = reinterpret_cast<const uint2*>(idx + base) + lane;
#pragma unroll
    for (int j = 0; j < kLaneUnroll; ++j) pre[j] = (g + j < ng) ? p[(size_t)(g + j) * 64] : make_uint2(0u, 0u);
  };
  // the first batch of task tn, if it is a lane task and its descriptor is in
  // the block loaded last
  auto issue_task = [&](int tn) {
    const int k = (tn - t0) & 63;
    if (tn < t1 && __builtin_amdgcn_readlane(my.x, k) == 0) {
      issue(__builtin_amdgcn_readlane(my.y, k), 0, __builtin_amdgcn_readlane(my.z, k) / kLaneGroup);
      have = true;
    }
  };
  auto issue_next = [&](int t) {
    if (((t + 1 - t0) & 63) != 0) issue_task(t + 1);
  };
  issue_task(t0);
  if (stage.sc) {   // convergence check of the preceding x/r update, under the slice copy
    __shared__ double red_s[kSliceWaves];
    double rz_unused;
    if (stage_update<kSliceBlock>(stage, red_s, rz_unused)) {
      __builtin_amdgcn_s_waitcnt(0);   // the slice copy lands before the workgroup ends
      return;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int t = t0; t < t1; ++t) {
    const int i = (t - t0) & 63;
    if (i == 0 && t != t0) {
      my = make_int4(0, 0, 0, 0);
      if (t + lane < t1) my = task[t + lane];
    }
    const int kind = __builtin_amdgcn_readlane(my.x, i);
    const int base = __builtin_amdgcn_readlane(my.y, i);
    const int len = __builtin_amdgcn_readlane(my.z, i);
    const int obase = __builtin_amdgcn_readlane(my.w, i);
    if (kind == 0) {
      // group g of lane l: entries 4 g .. 4 g + 3 in one 8-byte load
      T* o = out + obase + lane;
      T acc = T(0);
      const int ng = len / kLaneGroup;
      auto add = [&](unsigned e) {
        acc += vs[e & kLocalMask];
        if (e & kEndFlag) {
          *o = acc;
          o += 64;
          acc = T(0);
        }
      };
      for (int g = 0; g < ng; g += kLaneUnroll) {
        if (!have) issue(base, g, ng);
        uint2 q[kLaneUnroll];
#pragma unroll
        for (int j = 0; j < kLaneUnroll; ++j) q[j] = pre[j];
        have = false;
        if (g + kLaneUnroll < ng) {
          issue(base, g + kLaneUnroll, ng);
          have = true;
        } else {
          issue_next(t);
        }
        const int cnt = min(kLaneUnroll, ng - g);
#pragma unroll
        for (int j = 0; j < kLaneUnroll; ++j) {
          if (j < cnt) {
            add(q[j].x & 0xffffu);
            add(q[j].x >> 16);
            add(q[j].y & 0xffffu);
            add(q[j].y >> 16);
          }
        }
      }
    } else {
      issue_next(t);
      const uint4* p = reinterpret_cast<const uint4*>(idx) + base + lane;
      const int ng = len >> 4, nt = len & 15;
      T acc[4] = {T(0), T(0), T(0), T(0)};
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
            acc[(2 * h) & 3] += vs[wds[h] & kLocalMask];
            acc[(2 * h + 1) & 3] += vs[(wds[h] >> 16) & kLocalMask];
          }
        }
      }
      if (g < ng) {   // the rest (ng is the same in every lane): loads issued together
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
              acc[(2 * h) & 3] += vs[wds[h] & kLocalMask];
              acc[(2 * h + 1) & 3] += vs[(wds[h] >> 16) & kLocalMask];
            }
          }
        }
      }
      if (nt > 0) {   // tail: up to 8 groups of 64 entries, one 2-byte load per lane each
        const uint16_t* pt = idx + (size_t)base * 8 + (size_t)ng * 512 + lane;
        unsigned q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = (j < nt) ? (unsigned)pt[j * 64] : (unsigned)W;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < nt) acc[j & 3] += vs[q[j] & kLocalMask];
      }
      T s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) out[obase] = s;
    }
  }
}

// PASS only names the instantiation (0: rows of X, 1: columns of X, 2: the
// columns of X P), so a profiler reports the passes apart.
template <int PASS>
__global__ __launch_bounds__(kSliceBlock) void k_sell(const int* __restrict__ wrange,
                                                     const int* __restrict__ bslice,
                                                     const int4* __restrict__ task,
                                                     const uint16_t* __restrict__ idx,
                                                     const double* __restrict__ v, int gdim,
                                                     int W, double* __restrict__ out,
                                                     const int* done, StageArgs stage) {
  sell_body<double>(wrange, bslice, task, idx, v, gdim, W, out, done, stage);
}

// The passes of a valued X: every entry's FP64 value is streamed beside its
// index (the same positions, 0 for padding) and multiplies the LDS value.
// Lane tasks load 4 groups of 4 entries per batch (8-byte index loads and
// 16-byte value loads), wave tasks 2 groups of 8 entries per lane; the sums
// run in the same fixed orders as for 0/1 X.
constexpr int kLaneUnrollV = 4;
constexpr int kWaveUnrollV = 2;

template <int PASS>
__global__ __launch_bounds__(kSliceBlock) void k_sell_val(const int* __restrict__ wrange,
                                                         const int* __restrict__ bslice,
                                                         const int4* __restrict__ task,
                                                         const uint16_t* __restrict__ idx,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ v, int gdim, int W,
                                                         double* __restrict__ out, const int* done,
                                                         StageArgs stage) {
  if (is_done(done)) return;
  __shared__ __align__(16) double vs[kSliceRows + 1];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int t0 = wrange[blockIdx.x * (kSliceWaves + 1) + w];
  const int t1 = wrange[blockIdx.x * (kSliceWaves + 1) + w + 1];
  int4 my = make_int4(0, 0, 0, 0);
  if (t0 + lane < t1) my = task[t0 + lane];
  const int g0 = bslice[blockIdx.x] * W;
  fill_slice(vs, v + g0, min(W, gdim - g0));
  if (stage.sc) {   // convergence check of the preceding x/r update, under the slice copy
    __shared__ double red_s[kSliceWaves];
    double rz_unused;
    if (stage_update<kSliceBlock>(stage, red_s, rz_unused)) {
      __builtin_amdgcn_s_waitcnt(0);   // the slice copy lands before the workgroup ends
      return;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const double2 z2 = make_double2(0.0, 0.0);
  for (int t = t0; t < t1; ++t) {
    const int i = (t - t0) & 63;
    if (i == 0 && t != t0) {
      my = make_int4(0, 0, 0, 0);
      if (t + lane < t1) my = task[t + lane];
    }
    const int kind = __builtin_amdgcn_readlane(my.x, i);
    const int base = __builtin_amdgcn_readlane(my.y, i);
    const int len = __builtin_amdgcn_readlane(my.z, i);
    const int obase = __builtin_amdgcn_readlane(my.w, i);
    if (kind == 0) {
      // group g of lane l: entries 4 g .. 4 g + 3, indexes in one 8-byte
      // load, values in two 16-byte loads
      const uint2* p = reinterpret_cast<const uint2*>(idx + base) + lane;
      const double2* pv = reinterpret_cast<const double2*>(val + base) + 2 * lane;
      double* o = out + obase + lane;
      double acc = 0.0;
      const int ng = len / kLaneGroup;
      auto add = [&](unsigned e, double x) {
        acc += vs[e & kLocalMask] * x;
        if (e & kEndFlag) {
          *o = acc;
          o += 64;
          acc = 0.0;
        }
      };
      for (int g = 0; g < ng; g += kLaneUnrollV) {
        uint2 q[kLaneUnrollV];
        double2 a[kLaneUnrollV], b[kLaneUnrollV];
#pragma unroll
        for (int j = 0; j < kLaneUnrollV; ++j) {
          const bool in = g + j < ng;
          q[j] = in ? p[(size_t)(g + j) * 64] : make_uint2(0u, 0u);
          a[j] = in ? pv[(size_t)(g + j) * 128] : z2;
          b[j] = in ? pv[(size_t)(g + j) * 128 + 1] : z2;
        }
#pragma unroll
        for (int j = 0; j < kLaneUnrollV; ++j) {
          if (g + j < ng) {
            add(q[j].x & 0xffffu, a[j].x);
            add(q[j].x >> 16, a[j].y);
            add(q[j].y & 0xffffu, b[j].x);
            add(q[j].y >> 16, b[j].y);
          }
        }
      }
    } else {
      // groups of 512 entries: lane l reads 8 entries (one 16-byte index
      // load, four 16-byte value loads) of each, then 64-entry tail groups
      const uint4* p = reinterpret_cast<const uint4*>(idx) + base + lane;
      const double2* pv = reinterpret_cast<const double2*>(val + (size_t)base * 8) + 4 * lane;
      const int ng = len >> 4, nt = len & 15;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int g = 0; g < ng; g += kWaveUnrollV) {
        uint4 q[kWaveUnrollV];
        double2 x[kWaveUnrollV][4];
#pragma unroll
        for (int j = 0; j < kWaveUnrollV; ++j) {
          const bool in = g + j < ng;
          q[j] = in ? p[(size_t)(g + j) * 64] : make_uint4(0, 0, 0, 0);
#pragma unroll
          for (int h = 0; h < 4; ++h) x[j][h] = in ? pv[(size_t)(g + j) * 256 + h] : z2;
        }
#pragma unroll
        for (int j = 0; j < kWaveUnrollV; ++j) {
          if (g + j < ng) {
            const unsigned wds[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              acc[(2 * h) & 3] += vs[wds[h] & kLocalMask] * x[j][h].x;
              acc[(2 * h + 1) & 3] += vs[(wds[h] >> 16) & kLocalMask] * x[j][h].y;
            }
          }
        }
      }
      if (nt > 0) {   // tail: up to 8 groups of 64 entries, one entry per lane each
        const size_t tb = (size_t)base * 8 + (size_t)ng * 512 + lane;
        unsigned q[8];
        double x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          q[j] = (j < nt) ? (unsigned)idx[tb + j * 64] : (unsigned)W;
          x[j] = (j < nt) ? val[tb + j * 64] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < nt) acc[j & 3] += vs[q[j] & kLocalMask] * x[j];
      }
      double sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
      if (lane == 0) out[obase] = sum;
    }
  }
}

// The same passes over single-precision vectors (FP32 sums).
template <int PASS>
__global__ __launch_bounds__(kSliceBlock) void k_sell32(const int* __restrict__ wrange,
                                                       const int* __restrict__ bslice,
                                                       const int4* __restrict__ task,
                                                       const uint16_t* __restrict__ idx,
                                                       const float* __restrict__ v, int gdim,
                                                       int W, float* __restrict__ out,
                                                       const int* done, StageArgs stage) {
  sell_body<float>(wrange, bslice, task, idx, v, gdim, W, out, done, stage);
}

// segment s: t = sum of its partial sums, then the epilogue.  Segments of
// up to kReduceBatch pieces take one thread, which loads the positions and
// values of all pieces together and adds them in slice order; the longer
// ones (listed in lseg) take a whole wave each, on blocks of their own,
// lane i adding pieces i, i + 64, ... before a fixed butterfly.
constexpr int kReduceBatch = 16;

template <typename T>
__device__ inline T short_seg_sum(const T* __restrict__ part, const int* __restrict__ pos, int a, int z) {
  int pi[kReduceBatch];
#pragma unroll
  for (int j = 0; j < kReduceBatch; ++j) pi[j] = (a + j < z) ? pos[a + j] : -1;
  T pv[kReduceBatch];
#pragma unroll
  for (int j = 0; j < kReduceBatch; ++j) pv[j] = (pi[j] >= 0) ? part[pi[j]] : T(0);
  T t = T(0);
#pragma unroll
  for (int j = 0; j < kReduceBatch; ++j)
    if (a + j < z) t += pv[j];
  return t;
}

template <typename T>
__device__ inline T long_seg_sum(const T* __restrict__ part, const int* __restrict__ pos, int a, int z,
                                 int lane) {
  T t = T(0);
  for (int k = a + lane; k < z; k += 64) t += part[pos[k]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  return t;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_sell_reduce(const double* __restrict__ part,
                                                       const int* __restrict__ pos,
                                                       const int* __restrict__ sbase, int S,
                                                       const int* __restrict__ lseg, int nlong, int nlb,
                                                       Epi e, const int* done) {
  if (is_done(done)) return;
  double dot = 0.0;
  const int nsb = gridDim.x - nlb;   // the last nlb blocks take the long segments
  if ((int)blockIdx.x >= nsb) {
    for (int L = ((blockIdx.x - nsb) * kBlock + threadIdx.x) >> 6; L < nlong; L += nlb * (kBlock / 64)) {
      const int s = lseg[L];
      const double t = long_seg_sum(part, pos, sbase[s], sbase[s + 1], threadIdx.x & 63);
      if ((threadIdx.x & 63) == 0) seg_finish<MODE>(s, t, e, dot);
    }
  } else {
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += nsb * kBlock) {
      const int a = sbase[s], z = sbase[s + 1];
      if (z - a > kReduceBatch) continue;
      seg_finish<MODE>(s, short_seg_sum(part, pos, a, z), e, dot);
    }
  }
  if constexpr (has_dot<MODE>()) store_block_partial<kBlock>(dot, e.partials, blockIdx.x);
}

// Blocks of the segment reduction: up to 256 for the long segments, the
// rest (at least one) for the others; at most kMaxReduceBlocks in all.
static int sell_long_blocks(const SellPlan& sp) { return std::min(256, cdiv(sp.nlong, kBlock / 64)); }
int sell_reduce_grid(const SellPlan& sp) {
  const int nlb = sell_long_blocks(sp);
  return std::max(1, std::min(kMaxReduceBlocks - nlb, cdiv(sp.S, kBlock))) + nlb;
}

// Single-precision segment reduction: FP32 sums and epilogue, FP64 dot
// products (modes EPI_STORE, EPI_APPLY_DOT, EPI_RESID, EPI_POST; EPI_RESID
// stores its result widened to FP64 for the FP64 restriction).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_sell_reduce32(const float* __restrict__ part,
                                                         const int* __restrict__ pos,
                                                         const int* __restrict__ sbase, int S,
                                                         const int* __restrict__ lseg, int nlong, int nlb,
                                                         Epi32 e, const int* done) {
  if (is_done(done)) return;
  double dot = 0.0;
  const float lam = (float)e.lam, omega = (float)e.omega;
  auto finish = [&](int s, float t) {
    if constexpr (MODE == EPI_STORE) {
      e.out[s] = t;
    } else if constexpr (MODE == EPI_APPLY_DOT) {
      const float ps = e.p[s];
      const float q = t + lam * ps;
      e.out[s] = q;
      dot += (double)ps * (double)q;
    } else if constexpr (MODE == EPI_RESID) {
      e.out64[s] = (double)(e.r[s] - (t + lam * e.p[s]));
    } else if constexpr (MODE == EPI_POST) {
      const float e2 = e.p[s], rs = e.r[s];
      const float rho = rs - (t + lam * e2);
      const float zz = e2 + (omega * rho) / e.D[s];
      e.out[s] = zz;
      dot += (double)rs * (double)zz;
    }
  };
  const int nsb = gridDim.x - nlb;
  if ((int)blockIdx.x >= nsb) {
    for (int L = ((blockIdx.x - nsb) * kBlock + threadIdx.x) >> 6; L < nlong; L += nlb * (kBlock / 64)) {
      const int s = lseg[L];
      const float t = long_seg_sum(part, pos, sbase[s], sbase[s + 1], threadIdx.x & 63);
      if ((threadIdx.x & 63) == 0) finish(s, t);
    }
  } else {
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += nsb * kBlock) {
      const int a = sbase[s], z = sbase[s + 1];
      if (z - a > kReduceBatch) continue;
      finish(s, short_seg_sum(part, pos, a, z));
    }
  }
  if constexpr (MODE == EPI_APPLY_DOT || MODE == EPI_POST)
    store_block_partial<kBlock>(dot, e.partials, blockIdx.x);
}

int launch_sell32(const SellPlan& sp, float* part, const float* v, int mode, const Epi32& e,
                  const int* done, hipStream_t s, const StageArgs* stage) {
  StageArgs st{};
  if (stage) st = *stage;
  if (sp.nblk > 0) {
    if (sp.pass == 0)
      k_sell32<0><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, v, sp.gdim,
                                                 sp.W, part, done, st);
    else
      k_sell32<1><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, v, sp.gdim,
                                                 sp.W, part, done, st);
  } else if (stage) {
    launch_stage_update(*stage, s);
  }
  const int g = sell_reduce_grid(sp), nlb = sell_long_blocks(sp);
  switch (mode) {
    case EPI_STORE:
      k_sell_reduce32<EPI_STORE><<<g, kBlock, 0, s>>>(part, sp.pos, sp.sbase, sp.S, sp.lseg, sp.nlong,
                                                         nlb, e, done);
      return 0;
    case EPI_APPLY_DOT:
      k_sell_reduce32<EPI_APPLY_DOT><<<g, kBlock, 0, s>>>(part, sp.pos, sp.sbase, sp.S, sp.lseg, sp.nlong,
                                                             nlb, e, done);
      break;
    case EPI_RESID:
      k_sell_reduce32<EPI_RESID><<<g, kBlock, 0, s>>>(part, sp.pos, sp.sbase, sp.S, sp.lseg, sp.nlong,
                                                         nlb, e, done);
      return 0;
    case EPI_POST:
      k_sell_reduce32<EPI_POST><<<g, kBlock, 0, s>>>(part, sp.pos, sp.sbase, sp.S, sp.lseg, sp.nlong,
                                                        nlb, e, done);
      break;
    default:
      return 0;
  }
  return collapse_parts(e.partials, g, done, s);
}

template <int MODE>
static void sell_reduce_mode(const SellPlan& sp, const Epi& e, const int* done, hipStream_t s) {
  k_sell_reduce<MODE><<<sell_reduce_grid(sp), kBlock, 0, s>>>(sp.part, sp.pos, sp.sbase, sp.S, sp.lseg,
                                                              sp.nlong, sell_long_blocks(sp), e, done);
}

int launch_sell(const SellPlan& sp, const double* v, int mode, const Epi& e, const int* done,
                hipStream_t s, const StageArgs* stage, hipEvent_t mid) {
  StageArgs st{};
  if (stage) st = *stage;
  if (sp.nblk > 0) {
    if (sp.val)
      k_sell_val<1><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, sp.val, v,
                                                    sp.gdim, sp.W, sp.part, done, st);
    else if (sp.pass == 0)
      k_sell<0><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, v, sp.gdim,
                                               sp.W, sp.part, done, st);
    else
      k_sell<1><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, v, sp.gdim,
                                               sp.W, sp.part, done, st);
  } else if (stage) {
    launch_stage_update(*stage, s);
  }
  if (mid) (void)hipEventRecord(mid, s);
  switch (mode) {
    case EPI_STORE: sell_reduce_mode<EPI_STORE>(sp, e, done, s); break;
    case EPI_APPLY: sell_reduce_mode<EPI_APPLY>(sp, e, done, s); break;
    case EPI_APPLY_DOT: sell_reduce_mode<EPI_APPLY_DOT>(sp, e, done, s); break;
    case EPI_APPLY_DOT_P: sell_reduce_mode<EPI_APPLY_DOT_P>(sp, e, done, s); break;
    case EPI_RESID: sell_reduce_mode<EPI_RESID>(sp, e, done, s); break;
    case EPI_POST: sell_reduce_mode<EPI_POST>(sp, e, done, s); break;
    case EPI_POST_P: sell_reduce_mode<EPI_POST_P>(sp, e, done, s); break;
    case EPI_TRUE: sell_reduce_mode<EPI_TRUE>(sp, e, done, s); break;
    case EPI_SCALE: sell_reduce_mode<EPI_SCALE>(sp, e, done, s); break;
  }
  if (mode != EPI_APPLY_DOT && mode != EPI_APPLY_DOT_P && mode != EPI_POST && mode != EPI_POST_P &&
      mode != EPI_TRUE)
    return 0;
  return collapse_parts(e.partials, sell_reduce_grid(sp), done, s);
}

void launch_sell_gather(const SellPlan& sp, const double* v, hipStream_t s, const int* done) {
  if (sp.nblk == 0) return;
  const StageArgs st{};
  if (sp.val)
    k_sell_val<1><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, sp.val, v, sp.gdim,
                                                  sp.W, sp.part, done, st);
  else if (sp.pass == 0)
    k_sell<0><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, v, sp.gdim,
                                             sp.W, sp.part, done, st);
  else if (sp.pass == 2)
    k_sell<2><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, v, sp.gdim,
                                             sp.W, sp.part, done, st);
  else
    k_sell<1><<<sp.nblk, kSliceBlock, 0, s>>>(sp.wrange, sp.bslice, sp.task, sp.idx, v, sp.gdim,
                                             sp.W, sp.part, done, st);
}

void free_sell(SellPlan& sp) {
  if (sp.idx) (void)dev_free(sp.idx);
  if (sp.task) (void)dev_free(sp.task);
  if (sp.wrange) (void)dev_free(sp.wrange);
  if (sp.bslice) (void)dev_free(sp.bslice);
  if (sp.pos) (void)dev_free(sp.pos);
  if (sp.sbase) (void)dev_free(sp.sbase);
  if (sp.lseg) (void)dev_free(sp.lseg);
  if (sp.part) (void)dev_free(sp.part);
  if (sp.val) (void)dev_free(sp.val);
  sp = SellPlan{};
}

namespace {

struct Pair {
  int start, len;
};

// Lane-task builder state: indexes, tasks, output positions.
struct SellBuild {
  std::vector<uint16_t> idx;
  std::vector<double> val;   // valued X: values at the indexes' positions (0 for padding)
  bool valued = false;
  std::vector<int4> tasks;
  std::vector<long long> tcost;
  std::vector<int> tslice;
  std::vector<int> pos;      // per pair: output position
  int nout = 0;
};

// One lane task from a stack of layers of up to 64 pairs each: lane l takes
// the layer's l-th pair, padded with the zero entry to the layer's length
// llen[c] (its longest pair), and every lane's stream carries the end flag on
// the layer's last entry, so that the layer's 64 sums are stored together,
// at obase + 64 c + l.
void emit_layer_task(SellBuild& B, const std::vector<std::vector<int>>& layers,
                     const std::vector<int>& llen, const std::vector<Pair>& pairs,
                     const std::vector<int>& gidx, const std::vector<double>* gval, int g0, int W,
                     int r) {
  int m = 0;
  for (int L : llen) m += L;
  m = (m + kLaneGroup - 1) / kLaneGroup * kLaneGroup;
  const size_t base = B.idx.size();   // a multiple of 64: every task fills whole 64-entry rows
  B.idx.resize(base + (size_t)m * 64, (uint16_t)W);
  if (B.valued) B.val.resize(B.idx.size(), 0.0);
  auto at = [&](int k, int l) {
    return base + (size_t)(k / kLaneGroup) * 64 * kLaneGroup + (size_t)l * kLaneGroup + k % kLaneGroup;
  };
  const int obase = B.nout;
  int k0 = 0;
  for (size_t c = 0; c < layers.size(); ++c) {
    for (int l = 0; l < 64; ++l) {
      if (l < (int)layers[c].size()) {
        const Pair& pa = pairs[layers[c][l]];
        for (int e = 0; e < pa.len; ++e) {
          B.idx[at(k0 + e, l)] = (uint16_t)(gidx[pa.start + e] - g0);
          if (B.valued) B.val[at(k0 + e, l)] = (*gval)[pa.start + e];
        }
        B.pos[layers[c][l]] = obase + (int)c * 64 + l;
      }
      B.idx[at(k0 + llen[c] - 1, l)] |= (uint16_t)kEndFlag;
    }
    k0 += llen[c];
  }
  B.nout += (int)layers.size() * 64;
  B.tasks.push_back(make_int4(0, (int)base, m, obase));
  B.tcost.push_back((long long)m + 4);
  B.tslice.push_back(r);
}

}  // namespace

// Host-side construction from a segment-major pattern (ptr[S+1], gidx sorted
// inside every segment).  Setup only.
rr_status build_sell(SellPlan& sp, const std::vector<int>& ptr, const std::vector<int>& gidx,
                     int S, int gdim, int num_cu, hipStream_t s, int target_div,
                     const std::vector<double>* gval) {
  free_sell(sp);
  const int W = kSliceRows;
  const int R = std::max(1, cdiv(gdim, W));
  sp.S = S;
  sp.gdim = gdim;
  sp.W = W;
  sp.R = R;
  // nonempty (segment, slice) pairs in (segment, slice) order
  std::vector<Pair> pairs;
  std::vector<int> pslice;
  std::vector<int> pseg;
  pairs.reserve(ptr[S] / 2 + S);
  for (int q = 0; q < S; ++q) {
    int e = ptr[q];
    const int z = ptr[q + 1];
    while (e < z) {
      const int r = gidx[e] / W;
      int f = e;
      while (f < z && gidx[f] / W == r) ++f;
      pairs.push_back({e, f - e});
      pslice.push_back(r);
      pseg.push_back(q);
      e = f;
    }
  }
  sp.nslots = (int)pairs.size();
  const long long nnz = ptr[S];
  // lane streams of about `target` entries; pairs of (2, 4] target entries
  // are cut in two halves, each with its own partial sum; longer pairs get
  // wave tasks
  const int target = (int)std::min<long long>(
      64, std::max<long long>(8, nnz / std::max(1LL, (long long)num_cu * kSliceWaves * 64 *
                                                        std::max(1, target_div))));
  const int cmax = 2 * target;
  // pairs longer than hcap entries (a wave's mean share of the pass, in
  // whole 512-entry groups) become several wave tasks, so that no wave holds
  // one pair much longer than the others' work
  const int hcap = (int)std::max<long long>(
      1024, nnz / ((long long)std::max(1, num_cu) * kSliceWaves) / 512 * 512);
  std::vector<Pair> items;
  std::vector<int> islice;
  std::vector<int> sbase(S + 1, 0);
  items.reserve(pairs.size() + nnz / cmax + 1);
  for (size_t i = 0, q = 0; q <= (size_t)S; ++q) {
    sbase[q] = (int)items.size();
    if (q == (size_t)S) break;
    for (; i < pairs.size() && pseg[i] == (int)q; ++i) {
      const Pair pa = pairs[i];
      if (pa.len > hcap) {
        const int nc = cdiv(pa.len, hcap);
        const int step = cdiv(cdiv(pa.len, nc), 512) * 512;
        for (int a = 0; a < pa.len; a += step) {
          items.push_back({pa.start + a, std::min(step, pa.len - a)});
          islice.push_back(pslice[i]);
        }
        continue;
      }
      const int nc = (pa.len > cmax && pa.len <= 2 * cmax) ? 2 : 1;
      for (int c = 0; c < nc; ++c) {
        const int a = (int)((long long)pa.len * c / nc), b = (int)((long long)pa.len * (c + 1) / nc);
        items.push_back({pa.start + a, b - a});
        islice.push_back(pslice[i]);
      }
    }
  }
  pairs.swap(items);
  pslice.swap(islice);
  sp.nitems = (int)pairs.size();
  std::vector<std::vector<int>> small(R), heavy(R);
  for (int i = 0; i < (int)pairs.size(); ++i) (pairs[i].len > cmax ? heavy : small)[pslice[i]].push_back(i);
  SellBuild B;
  B.valued = gval != nullptr;
  B.pos.assign(pairs.size(), -1);
  const uint16_t pad = (uint16_t)W;   // index of the zero entry
  auto by_len_desc = [&](int a, int b) {
    return pairs[a].len != pairs[b].len ? pairs[a].len > pairs[b].len : a < b;
  };
  for (int r = 0; r < R; ++r) {
    const int g0 = r * W;
    for (int i : heavy[r]) {
      while (B.idx.size() % 8) B.idx.push_back(pad);
      if (B.valued) B.val.resize(B.idx.size(), 0.0);
      const int base16 = (int)(B.idx.size() / 8);
      const int len = pairs[i].len;
      const int ng = len / 512;                  // 512-entry groups (16-byte loads)
      const int nt = cdiv(len - ng * 512, 64);   // 64-entry tail groups (2-byte loads)
      for (int k = 0; k < ng * 512 + nt * 64; ++k) {
        B.idx.push_back(k < len ? (uint16_t)(gidx[pairs[i].start + k] - g0) : pad);
        if (B.valued) B.val.push_back(k < len ? (*gval)[pairs[i].start + k] : 0.0);
      }
      B.pos[i] = B.nout++;
      B.tasks.push_back(make_int4(1, base16, ng * 16 + nt, B.pos[i]));
      B.tcost.push_back((long long)ng * 8 + nt + 8);
      B.tslice.push_back(r);
    }
  }
  // short pairs, longest first, in layers of 64; the layers, longest first,
  // go to the least loaded of ntask stacks, one lane task each.  Returns the
  // number of tasks, adds their cost to *cost and emits them if asked.
  auto pack_small = [&](int r, int ntask, bool emit, long long* cost) -> int {
    const std::vector<int>& sm = small[r];
    const int nlay = cdiv((int)sm.size(), 64);
    std::vector<std::vector<int>> stack(ntask);
    std::vector<long long> load(ntask, 0);
    using Item = std::pair<long long, int>;   // (load, stack)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int k = 0; k < ntask; ++k) heap.push({0, k});
    for (int c = 0; c < nlay; ++c) {
      const Item it = heap.top();
      heap.pop();
      stack[it.second].push_back(c);
      load[it.second] += pairs[sm[64 * c]].len;
      heap.push({load[it.second], it.second});
    }
    int cnt = 0;
    for (int k = 0; k < ntask; ++k) {
      if (stack[k].empty()) continue;
      ++cnt;
      *cost += (load[k] + kLaneGroup - 1) / kLaneGroup * kLaneGroup + 4;
      if (!emit) continue;
      std::vector<std::vector<int>> layers;
      std::vector<int> llen;
      for (int c : stack[k]) {
        layers.emplace_back(sm.begin() + 64 * c, sm.begin() + std::min<size_t>(sm.size(), 64 * c + 64));
        llen.push_back(pairs[sm[64 * c]].len);
      }
      emit_layer_task(B, layers, llen, pairs, gidx, gval, r * W, W, r);
    }
    return cnt;
  };
  std::vector<long long> ltot(R, 0), scost(R, 0);
  std::vector<int> lntask(R, 0), tcount(R, 0), nlay(R, 0);
  for (int r = 0; r < R; ++r) {
    std::vector<int>& sm = small[r];
    if (sm.empty()) continue;
    std::sort(sm.begin(), sm.end(), by_len_desc);
    nlay[r] = cdiv((int)sm.size(), 64);
    for (int c = 0; c < nlay[r]; ++c) ltot[r] += pairs[sm[64 * c]].len;
    lntask[r] = (int)std::min<long long>(nlay[r], std::max<long long>(1, (ltot[r] + target - 1) / target));
    tcount[r] += pack_small(r, lntask[r], false, &scost[r]);
  }
  // workgroups: each slice gets a share of about num_cu workgroups by cost;
  // its tasks go, heaviest first, to the least loaded wave of its workgroups
  long long total = 0;
  for (size_t t = 0; t < B.tasks.size(); ++t) {
    scost[B.tslice[t]] += B.tcost[t];
    tcount[B.tslice[t]]++;
  }
  for (int r = 0; r < R; ++r) total += scost[r];
  std::vector<int> nb(R, 0);
  {
    std::vector<std::pair<double, int>> frac;
    int used = 0;
    for (int r = 0; r < R; ++r) {
      if (scost[r] == 0) continue;
      const double share = (double)scost[r] / (double)total * num_cu;
      nb[r] = std::max(1, (int)share);
      used += nb[r];
      frac.push_back({share - (int)share, r});
    }
    std::sort(frac.begin(), frac.end(), [](auto& a, auto& b) { return a.first > b.first; });
    for (size_t k = 0; k < frac.size() && used < num_cu; ++k, ++used) nb[frac[k].second]++;
  }
  // the short pairs of every slice are re-stacked so that its task count is
  // a whole multiple of its waves, if that changes their stacks' height by
  // at most a fourth (fewer, taller stacks when the count is a little above
  // a multiple; more, lower ones of at least 8 entries when the slice has
  // idle waves): a wave with one task more than the others would set the
  // pass's time
  for (int r = 0; r < R; ++r) {
    if (small[r].empty()) continue;
    const int nbin = nb[r] * kSliceWaves;
    int nt = lntask[r];
    const int T = tcount[r];
    if (T > nbin) {
      const int excess = T - T / nbin * nbin;
      if (4 * (nt - excess) >= 3 * nt && nt - excess >= 1) nt -= excess;
    } else if (T < nbin) {
      nt = (int)std::max<long long>(nt, std::min<long long>({(long long)nt + (nbin - T), ltot[r] / 8,
                                                             (long long)nlay[r]}));
    }
    long long unused = 0;
    pack_small(r, nt, true, &unused);
  }
  std::vector<std::vector<int>> stasks(R);
  for (size_t t = 0; t < B.tasks.size(); ++t) stasks[B.tslice[t]].push_back((int)t);
  std::vector<int4> tasks_sorted;
  std::vector<int> wrange, bslice;
  tasks_sorted.reserve(B.tasks.size());
  for (int r = 0; r < R; ++r) {
    if (nb[r] == 0) continue;
    const int nbin = nb[r] * kSliceWaves;
    std::vector<int>& ts = stasks[r];
    std::stable_sort(ts.begin(), ts.end(), [&](int a, int b) { return B.tcost[a] > B.tcost[b]; });
    std::vector<std::vector<int>> bins(nbin);
    using Item = std::pair<long long, int>;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int k = 0; k < nbin; ++k) heap.push({0, k});
    for (int t : ts) {
      const Item it = heap.top();
      heap.pop();
      bins[it.second].push_back(t);
      heap.push({it.first + B.tcost[t], it.second});
    }
    for (int b = 0; b < nb[r]; ++b) {
      bslice.push_back(r);
      for (int w = 0; w < kSliceWaves; ++w) {
        wrange.push_back((int)tasks_sorted.size());
        for (int t : bins[b * kSliceWaves + w]) tasks_sorted.push_back(B.tasks[t]);
      }
      wrange.push_back((int)tasks_sorted.size());
    }
  }
  while (B.idx.size() % 8) B.idx.push_back(pad);
  if (B.idx.empty()) B.idx.resize(8, pad);
  if (B.valued) B.val.resize(B.idx.size(), 0.0);
  // the kernel trusts the plan: check every access it will make
  for (const int4& t : tasks_sorted) {
    const size_t n16 = B.idx.size();
    bool ok;
    if (t.x == 0)
      ok = t.z >= 1 && t.z % kLaneGroup == 0 && t.y % kLaneGroup == 0 &&
           (size_t)t.y + (size_t)t.z * 64 <= n16 && t.w >= 0 && t.w + 63 < B.nout;
    else
      ok = t.z >= 1 && (t.z & 15) <= 8 &&
           (size_t)t.y * 8 + (size_t)(t.z >> 4) * 512 + (size_t)(t.z & 15) * 64 <= n16 &&
           t.w >= 0 && t.w < B.nout;
    if (!ok) return fail(RR_ERR_DEVICE, "internal: SELL plan out of range");
  }
  for (uint16_t q : B.idx)
    if ((q & kLocalMask) > (unsigned)W) return fail(RR_ERR_DEVICE, "internal: SELL index out of range");
  for (const int4& t : tasks_sorted) {   // lane l's c-th output goes to t.w + 64 c + l
    if (t.x != 0) continue;
    for (int l = 0; l < 64; ++l) {
      int c = 0;
      for (int k = 0; k < t.z; ++k)
        if (B.idx[t.y + (size_t)(k / kLaneGroup) * 64 * kLaneGroup + (size_t)l * kLaneGroup +
                  k % kLaneGroup] & kEndFlag)
          ++c;
      if (c > 0 && t.w + 64 * (c - 1) + l >= B.nout)
        return fail(RR_ERR_DEVICE, "internal: SELL output out of range");
    }
  }
  for (int p : B.pos)
    if (p < 0 || p >= B.nout) return fail(RR_ERR_DEVICE, "internal: SELL output position missing");
  sp.nblk = (int)bslice.size();
  sp.ntask = (int)tasks_sorted.size();
  sp.nout = B.nout;
  RR_HIP(dmalloc(&sp.idx, sizeof(uint16_t) * B.idx.size()));
  RR_HIP(dmalloc(&sp.task, sizeof(int4) * std::max<size_t>(1, tasks_sorted.size())));
  RR_HIP(dmalloc(&sp.wrange, sizeof(int) * std::max<size_t>(1, wrange.size())));
  RR_HIP(dmalloc(&sp.bslice, sizeof(int) * std::max<size_t>(1, bslice.size())));
  RR_HIP(dmalloc(&sp.pos, sizeof(int) * std::max<size_t>(1, B.pos.size())));
  RR_HIP(dmalloc(&sp.sbase, sizeof(int) * sbase.size()));
  std::vector<int> lseg;
  for (int q = 0; q < S; ++q)
    if (sbase[q + 1] - sbase[q] > kReduceBatch) lseg.push_back(q);
  sp.nlong = (int)lseg.size();
  RR_HIP(dmalloc(&sp.lseg, sizeof(int) * std::max<size_t>(1, lseg.size())));
  if (!lseg.empty())
    RR_HIP(hipMemcpyAsync(sp.lseg, lseg.data(), sizeof(int) * lseg.size(), hipMemcpyHostToDevice, s));
  RR_HIP(dmalloc(&sp.part, sizeof(double) * std::max(1, sp.nout)));
  RR_HIP(hipMemcpyAsync(sp.idx, B.idx.data(), sizeof(uint16_t) * B.idx.size(), hipMemcpyHostToDevice, s));
  if (!tasks_sorted.empty())
    RR_HIP(hipMemcpyAsync(sp.task, tasks_sorted.data(), sizeof(int4) * tasks_sorted.size(),
                          hipMemcpyHostToDevice, s));
  if (!wrange.empty())
    RR_HIP(hipMemcpyAsync(sp.wrange, wrange.data(), sizeof(int) * wrange.size(), hipMemcpyHostToDevice, s));
  if (!bslice.empty())
    RR_HIP(hipMemcpyAsync(sp.bslice, bslice.data(), sizeof(int) * bslice.size(), hipMemcpyHostToDevice, s));
  if (!B.pos.empty())
    RR_HIP(hipMemcpyAsync(sp.pos, B.pos.data(), sizeof(int) * B.pos.size(), hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(sp.sbase, sbase.data(), sizeof(int) * sbase.size(), hipMemcpyHostToDevice, s));
  if (B.valued) {
    RR_HIP(dmalloc(&sp.val, sizeof(double) * B.val.size()));
    RR_HIP(hipMemcpyAsync(sp.val, B.val.data(), sizeof(double) * B.val.size(), hipMemcpyHostToDevice, s));
  }
  RR_HIP(hipStreamSynchronize(s));
  sp.idx_bytes = (long long)B.idx.size() * 2 + (long long)B.val.size() * 8;
  return RR_OK;
}

rr_status build_xp_plan(SellPlan& xp, const std::vector<int>& rp, const std::vector<int>& ci,
                        const std::vector<int>& lab, int N, int FC, int num_cu, int div, hipStream_t s) {
  free_sell(xp);
  const int nnz = rp[N];
  // cluster-major lists of X's entries: one pass over the rows in order
  // leaves every cluster's rows ascending, as the slicing needs
  std::vector<int> ptr(FC + 1, 0), rows(std::max(1, nnz));
  for (int e = 0; e < nnz; ++e) {
    const int c = lab[ci[e]];
    if (c < 0 || c >= FC) return fail(RR_ERR_DEVICE, "internal: label out of range");
    ++ptr[c + 1];
  }
  for (int c = 0; c < FC; ++c) ptr[c + 1] += ptr[c];
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int i = 0; i < N; ++i)
    for (int e = rp[i]; e < rp[i + 1]; ++e) rows[fill[lab[ci[e]]]++] = i;
  RR_TRY(build_sell(xp, ptr, rows, FC, N, num_cu, s, div, nullptr));
  xp.pass = 2;
  return RR_OK;
}

// Mean time of `reps` back-to-back launches of a pass (gather + reduction).
static rr_status time_pass(const SellPlan& sp, const double* v, double* out, int reps,
                           hipStream_t s, float* ms) {
  hipEvent_t a, b;
  RR_HIP(hipEventCreate(&a));
  RR_HIP(hipEventCreate(&b));
  Epi e{};
  e.out = out;
  launch_sell(sp, v, EPI_STORE, e, nullptr, s);
  RR_HIP(hipEventRecord(a, s));
  for (int i = 0; i < reps; ++i) launch_sell(sp, v, EPI_STORE, e, nullptr, s);
  RR_HIP(hipEventRecord(b, s));
  RR_HIP(hipEventSynchronize(b));
  RR_HIP(hipEventElapsedTime(ms, a, b));
  *ms /= reps;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return RR_OK;
}

// Mean time of `reps` back-to-back launches of the row pass.
static rr_status time_rows(const RowPlan& rp, const double* v, double* out, int reps, hipStream_t s,
                           float* ms) {
  hipEvent_t a, b;
  RR_HIP(hipEventCreate(&a));
  RR_HIP(hipEventCreate(&b));
  launch_rows(rp, v, out, nullptr, nullptr, s);
  RR_HIP(hipEventRecord(a, s));
  for (int i = 0; i < reps; ++i) launch_rows(rp, v, out, nullptr, nullptr, s);
  RR_HIP(hipEventRecord(b, s));
  RR_HIP(hipEventSynchronize(b));
  RR_HIP(hipEventElapsedTime(ms, a, b));
  *ms /= reps;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return RR_OK;
}

namespace {
// tuned (lanes per row, column lane-stream divisor) per shape bucket (log2 of N, F, nnz) and device
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune_cache;
}

rr_status build_sell_plans(Sparse& X, hipStream_t s, int autotune, SellTuning* tuned) {
  if (!X.binary && (X.N == 0 || X.nnz == 0)) return RR_OK;   // no entries: the generic kernels
  std::vector<int> rp(X.N + 1), ci(std::max(X.nnz, 1)), cp(X.F + 1), ri(std::max(X.nnz, 1));
  std::vector<double> rv, cv;   // valued X: CSR and CSC values
  RR_HIP(hipMemcpyAsync(rp.data(), X.row_ptr, sizeof(int) * (X.N + 1), hipMemcpyDeviceToHost, s));
  RR_HIP(hipMemcpyAsync(cp.data(), X.col_ptr, sizeof(int) * (X.F + 1), hipMemcpyDeviceToHost, s));
  if (X.nnz) {
    RR_HIP(hipMemcpyAsync(ci.data(), X.col_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToHost, s));
    RR_HIP(hipMemcpyAsync(ri.data(), X.row_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToHost, s));
  }
  if (!X.binary) {
    rv.resize(X.nnz);
    cv.resize(X.nnz);
    RR_HIP(hipMemcpyAsync(rv.data(), X.val, sizeof(double) * X.nnz, hipMemcpyDeviceToHost, s));
    RR_HIP(hipMemcpyAsync(cv.data(), X.cval, sizeof(double) * X.nnz, hipMemcpyDeviceToHost, s));
  }
  const std::vector<double>* rvp = X.binary ? nullptr : &rv;
  const std::vector<double>* cvp = X.binary ? nullptr : &cv;
  RR_HIP(hipStreamSynchronize(s));
  // defaults: two lanes per row once rows average 16 entries or more, four
  // from 64, eight from 256
  int lanes = 1, div_cols = 2;
  for (int t = 16; lanes < 8 && X.N > 0 && (long long)X.nnz >= (long long)t * X.N; t *= 4) lanes *= 2;
  if (autotune) {
    int dev = 0;
    RR_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    RR_HIP(hipGetDeviceProperties(&prop, dev));
    auto lg = [](long long v) { int b = 0; while ((1LL << b) < v) ++b; return b; };
    const std::string key = std::string(prop.gcnArchName) + ":" + std::to_string(lg(X.N)) + ":" +
                            std::to_string(lg(X.F)) + ":" + std::to_string(lg(X.nnz)) +
                            (X.binary ? ":01" : ":fp64");
    bool hit = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        lanes = it->second.first;
        div_cols = it->second.second;
        hit = true;
      }
    }
    if (tuned) tuned->cached = hit ? 1 : 0;
    if (!hit) {
      // build every candidate plan, time them in interleaved rounds on a
      // vector of ones (best round of each) and keep the fastest; a larger
      // candidate must win by 3 % to replace a smaller one
      double *v = nullptr, *out = nullptr;
      const int nmax = std::max(X.N, X.F);
      RR_HIP(dmalloc(&v, sizeof(double) * nmax));
      RR_HIP(dmalloc(&out, sizeof(double) * nmax));
      launch_fill(v, 1.0, nmax, s);
      // lanes per row: 1, 2, 4, and 8 and 16 for rows of 64 entries or more
      // on average (few long rows need more lanes than layers to fill the
      // chip); column lane-stream divisors: 1, 2, 4
      constexpr int kCandMax = 5, kCandCols = 3, kRounds = 5;
      const int cand[kCandMax] = {1, 2, 4, 8, 16};
      const int ncr = (X.N > 0 && (long long)X.nnz >= 64LL * X.N) ? 5 : 3;
      RowPlan rplans[kCandMax];
      SellPlan cplans[kCandCols];
      float best[2][kCandMax];
      rr_status st = RR_OK;
      for (int c = 0; c < kCandMax && st == RR_OK; ++c) {
        best[0][c] = best[1][c] = 1e30f;
        if (c < ncr) st = build_rows(rplans[c], rp, ci, X.N, X.F, X.num_cu, cand[c], s, rvp);
        if (st == RR_OK && c < kCandCols) {
          st = build_sell(cplans[c], cp, ri, X.F, X.N, X.num_cu, s, cand[c], cvp);
          cplans[c].pass = 1;
        }
      }
      for (int round = 0; round < kRounds && st == RR_OK; ++round)
        for (int c = 0; c < kCandMax && st == RR_OK; ++c) {
          float ms = 0.f;
          if (c < ncr) {
            st = time_rows(rplans[c], v, out, 4, s, &ms);
            best[0][c] = std::min(best[0][c], ms);
          }
          if (st == RR_OK && c < kCandCols) {
            st = time_pass(cplans[c], v, out, 4, s, &ms);
            best[1][c] = std::min(best[1][c], ms);
          }
        }
      for (int c = 0; c < kCandMax; ++c) {
        free_rows(rplans[c]);
        if (c < kCandCols) free_sell(cplans[c]);
      }
      if (st == RR_OK) {
        int pick[2] = {0, 0};
        for (int pass = 0; pass < 2; ++pass)
          for (int c = 1; c < (pass == 0 ? ncr : kCandCols); ++c)
            if (best[pass][c] < 0.97f * best[pass][pick[pass]]) pick[pass] = c;
        lanes = cand[pick[0]];
        div_cols = cand[pick[1]];
        if (tuned) {
          for (int pass = 0; pass < 2; ++pass)
            for (int c = 0; c < (pass == 0 ? ncr : kCandCols) && tuned->n < 8; ++c) {
              tuned->cand_div[tuned->n] = cand[c];
              tuned->cand_pass[tuned->n] = pass;
              tuned->cand_ms[tuned->n] = best[pass][c];
              tuned->n++;
            }
        }
      }
      (void)dev_free(v);
      (void)dev_free(out);
      RR_TRY(st);
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = {lanes, div_cols};
    }
  }
  if (tuned) {
    tuned->div_rows = lanes;
    tuned->div_cols = div_cols;
  }
  RR_TRY(build_rows(X.rows, rp, ci, X.N, X.F, X.num_cu, lanes, s, rvp));
  RR_TRY(build_sell(X.sell_csc, cp, ri, X.F, X.N, X.num_cu, s, div_cols, cvp));
  X.sell_csc.pass = 1;
  X.sliced = true;
  return RR_OK;
}

}  // namespace rr
