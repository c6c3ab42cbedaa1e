// Row pass of the operator for 0/1 matrices, u = X v (u_i = sum of v_j over
// the columns j of row i), in one kernel with no partial sums.
//
// The features are numbered by descending column count (the library's
// popularity order), so the first W = 16384 features carry most entries of
// every row (88 % on the 200,000 x 100,000 Zipf(1.1) workload).  Every
// workgroup copies v[0, W) into LDS once (128 KB of FP64, plus one zero
// entry for padding) and sums a row's "hot" entries from there; the row's
// remaining "cold" entries are gathered from v in global memory, where the
// few hundred KB of cold features stay resident in L2.  A row is finished
// by its own lanes, so u is written once per row with no partial sums and no
// second kernel (the sliced pass over all features wrote one partial per
// (row, slice) pair and needed a reduction kernel).
//
// Layout: rows are taken in order, 64 / L rows per layer (L lanes per row).
// Lane l of a layer serves row 64 c / L + l / L and takes every L-th hot and
// every L-th cold entry of it (entry k of the row goes to lane k mod L).  A
// layer holds two lane-interleaved streams padded to the layer's longest
// lane: hot uint16 local indexes (entry k of lane l at hoff + 256 (k / 4) +
// 4 l + k % 4, so each 8-byte load of 4 entries reads 512 consecutive bytes
// per wave; padding = W, the zero entry) and cold int32 feature indexes
// (the same interleave, 16-byte loads; padding = -1).  The lanes of a row add
// their sums in a fixed butterfly, so results are bitwise reproducible.
//
// A valued X streams each entry's FP64 value beside its index (hval, cval:
// the same positions, 0 for padding; 16-byte loads of two values), so the
// LDS slice serves the value-weighted sums as it serves the 0/1 ones.
#include <algorithm>
#include <climits>

#include "rr_device.h"

namespace rr {

constexpr int kHotBatch = 8;    // 8-byte hot index loads (4 entries each) per batch
constexpr int kColdBatch = 2;   // 16-byte cold index loads (4 entries each) per batch

// PU (FP64 only): v holds z and u holds X p of the previous direction; the
// pass writes u = X z + beta u, the new direction's X p, with the PCG
// update's beta = <r,z>_new / sc->rz (0 while sc->rz is 0: the first
// direction; u is then not read), <r,z>_new the sum of pu.parts[0, pu.n).
// Every workgroup adds the partials itself while its slice copy is in
// flight; workgroup 0 stores beta and <r,z>_new, and a non-finite or
// non-positive <r,z>_new ends the solve as a breakdown.
template <typename T, int L, bool PU = false>
__global__ __launch_bounds__(kSliceBlock) void k_rows(int nlayer, int N, const int4* __restrict__ lay,
                                                      const uint16_t* __restrict__ hidx,
                                                      const int* __restrict__ cidx,
                                                      const T* __restrict__ v, int F, T* __restrict__ u,
                                                      const double* __restrict__ scale, const int* done,
                                                      StageArgs stage, PUpd pu = PUpd{}) {
  static_assert(!PU || sizeof(T) == 8, "the folded direction update is FP64");
  if (is_done(done)) return;
  __shared__ __align__(16) T vs[kSliceRows + 1];
  constexpr unsigned kPad = (unsigned)kSliceRows | ((unsigned)kSliceRows << 16);
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * kSliceWaves;
  int c = blockIdx.x * kSliceWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int4 d = make_int4(0, 0, 0, 0);
  uint2 hq[kHotBatch];
  int4 cq[kColdBatch];
  // the first batch of hot and cold indexes of layer c
  auto load_first = [&]() {
    d = lay[c];
    const uint2* hp = reinterpret_cast<const uint2*>(hidx + d.x) + lane;
    const int4* cp = reinterpret_cast<const int4*>(cidx + d.z) + lane;
#pragma unroll
    for (int j = 0; j < kHotBatch; ++j) hq[j] = (4 * j < d.y) ? hp[j * 64] : make_uint2(kPad, kPad);
#pragma unroll
    for (int j = 0; j < kColdBatch; ++j) cq[j] = (4 * j < d.w) ? cp[j * 64] : make_int4(-1, -1, -1, -1);
  };
  bool have = c < nlayer;
  if (have) load_first();   // in flight during the slice copy
  fill_slice(vs, v, min(kSliceRows, F));
  T beta = T(0);
  if constexpr (PU) {   // beta under the slice copy
    __shared__ double red_p[kSliceWaves];
    const double rz_new = sum_parts<kSliceBlock>(pu.parts, pu.n, red_p);
    if (!finite_pos(rz_new)) {   // the same value in every thread of every workgroup
      if (is_block0_lead()) {
        pu.sc->status = RR_ERR_BREAKDOWN;
        pu.sc->done = 1;
      }
      __builtin_amdgcn_s_waitcnt(0);   // the slice copy lands before the workgroup ends
      return;
    }
    const double rz_old = pu.sc->rz;
    beta = rz_old == 0.0 ? 0.0 : rz_new / rz_old;
    if (is_block0_lead()) {
      pu.sc->rz_next = rz_new;
      pu.sc->beta = beta;
    }
  }
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
  for (; c < nlayer; c += nw) {
    if (!have) load_first();
    have = false;
    // cold entries of the first batch: gathers from global memory, issued
    // before the LDS sums
    T cv[4 * kColdBatch];
#pragma unroll
    for (int j = 0; j < kColdBatch; ++j) {
      cv[4 * j + 0] = cq[j].x >= 0 ? v[cq[j].x] : T(0);
      cv[4 * j + 1] = cq[j].y >= 0 ? v[cq[j].y] : T(0);
      cv[4 * j + 2] = cq[j].z >= 0 ? v[cq[j].z] : T(0);
      cv[4 * j + 3] = cq[j].w >= 0 ? v[cq[j].w] : T(0);
    }
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    auto add_hot = [&]() {
#pragma unroll
      for (int j = 0; j < kHotBatch; ++j) {
        a0 += vs[hq[j].x & 0xffffu];
        a1 += vs[hq[j].x >> 16];
        a2 += vs[hq[j].y & 0xffffu];
        a3 += vs[hq[j].y >> 16];
      }
    };
    add_hot();
    for (int g = 4 * kHotBatch; g < d.y; g += 4 * kHotBatch) {   // longer rows: further batches
      const uint2* hp = reinterpret_cast<const uint2*>(hidx + d.x) + (g / 4) * 64 + lane;
#pragma unroll
      for (int j = 0; j < kHotBatch; ++j) hq[j] = (g + 4 * j < d.y) ? hp[j * 64] : make_uint2(kPad, kPad);
      add_hot();
    }
    T cs = T(0);
#pragma unroll
    for (int k = 0; k < 4 * kColdBatch; ++k) cs += cv[k];
    for (int g = 4 * kColdBatch; g < d.w; g += 4 * kColdBatch) {
      const int4* cp = reinterpret_cast<const int4*>(cidx + d.z) + (g / 4) * 64 + lane;
#pragma unroll
      for (int j = 0; j < kColdBatch; ++j) cq[j] = (g + 4 * j < d.w) ? cp[j * 64] : make_int4(-1, -1, -1, -1);
#pragma unroll
      for (int j = 0; j < kColdBatch; ++j) {
        cv[4 * j + 0] = cq[j].x >= 0 ? v[cq[j].x] : T(0);
        cv[4 * j + 1] = cq[j].y >= 0 ? v[cq[j].y] : T(0);
        cv[4 * j + 2] = cq[j].z >= 0 ? v[cq[j].z] : T(0);
        cv[4 * j + 3] = cq[j].w >= 0 ? v[cq[j].w] : T(0);
      }
#pragma unroll
      for (int k = 0; k < 4 * kColdBatch; ++k) cs += cv[k];
    }
    T sum = ((a0 + a1) + (a2 + a3)) + cs;
    if constexpr (L >= 2) sum += __shfl_xor(sum, 1, 64);
    if constexpr (L >= 4) sum += __shfl_xor(sum, 2, 64);
    if constexpr (L >= 8) sum += __shfl_xor(sum, 4, 64);
    if constexpr (L >= 16) sum += __shfl_xor(sum, 8, 64);
    const int row = c * (64 / L) + lane / L;
    if ((lane & (L - 1)) == 0 && row < N) {
      T o = scale ? (T)((double)sum * scale[row]) : sum;
      if constexpr (PU) {
        if (beta != T(0)) o += beta * u[row];
      }
      u[row] = o;
    }
  }
}

// u_i = sum over row i of X_ij v_j for a valued X: the value streams are read
// beside the index streams (batches of 4 hot and 2 cold index loads with
// their values, all issued before the sums).
constexpr int kHotBatchV = 4;
constexpr int kColdBatchV = 2;

template <int L>
__global__ __launch_bounds__(kSliceBlock) void k_rows_val(int nlayer, int N, const int4* __restrict__ lay,
                                                          const uint16_t* __restrict__ hidx,
                                                          const double* __restrict__ hval,
                                                          const int* __restrict__ cidx,
                                                          const double* __restrict__ cval,
                                                          const double* __restrict__ v, int F,
                                                          double* __restrict__ u,
                                                          const double* __restrict__ scale, const int* done,
                                                          StageArgs stage) {
  if (is_done(done)) return;
  __shared__ __align__(16) double vs[kSliceRows + 1];
  constexpr unsigned kPad = (unsigned)kSliceRows | ((unsigned)kSliceRows << 16);
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * kSliceWaves;
  int c = blockIdx.x * kSliceWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  fill_slice(vs, v, min(kSliceRows, F));
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
  for (; c < nlayer; c += nw) {
    const int4 d = lay[c];
    // entry k of this lane: index at offset 256 (k / 4) + 4 lane + k % 4 of
    // the layer's stream, value at the same offset of the value stream
    const uint2* hp = reinterpret_cast<const uint2*>(hidx + d.x) + lane;
    const double2* hv = reinterpret_cast<const double2*>(hval + d.x) + 2 * lane;
    const int4* cp = reinterpret_cast<const int4*>(cidx + d.z) + lane;
    const double2* cv = reinterpret_cast<const double2*>(cval + d.z) + 2 * lane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int g = 0; g < d.y; g += 4 * kHotBatchV) {
      uint2 q[kHotBatchV];
      double2 w0[kHotBatchV], w1[kHotBatchV];
#pragma unroll
      for (int j = 0; j < kHotBatchV; ++j) {
        const int G = g / 4 + j;
        const bool in = 4 * G < d.y;
        q[j] = in ? hp[G * 64] : make_uint2(kPad, kPad);
        w0[j] = in ? hv[G * 128] : z2;
        w1[j] = in ? hv[G * 128 + 1] : z2;
      }
#pragma unroll
      for (int j = 0; j < kHotBatchV; ++j) {
        a0 += vs[q[j].x & 0xffffu] * w0[j].x;
        a1 += vs[q[j].x >> 16] * w0[j].y;
        a2 += vs[q[j].y & 0xffffu] * w1[j].x;
        a3 += vs[q[j].y >> 16] * w1[j].y;
      }
    }
    double cs = 0.0;
    for (int g = 0; g < d.w; g += 4 * kColdBatchV) {
      int4 q[kColdBatchV];
      double2 w0[kColdBatchV], w1[kColdBatchV];
#pragma unroll
      for (int j = 0; j < kColdBatchV; ++j) {
        const int G = g / 4 + j;
        const bool in = 4 * G < d.w;
        q[j] = in ? cp[G * 64] : make_int4(-1, -1, -1, -1);
        w0[j] = in ? cv[G * 128] : z2;
        w1[j] = in ? cv[G * 128 + 1] : z2;
      }
      double x[4 * kColdBatchV];
#pragma unroll
      for (int j = 0; j < kColdBatchV; ++j) {
        x[4 * j + 0] = q[j].x >= 0 ? v[q[j].x] * w0[j].x : 0.0;
        x[4 * j + 1] = q[j].y >= 0 ? v[q[j].y] * w0[j].y : 0.0;
        x[4 * j + 2] = q[j].z >= 0 ? v[q[j].z] * w1[j].x : 0.0;
        x[4 * j + 3] = q[j].w >= 0 ? v[q[j].w] * w1[j].y : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4 * kColdBatchV; ++k) cs += x[k];
    }
    double sum = ((a0 + a1) + (a2 + a3)) + cs;
    if constexpr (L >= 2) sum += __shfl_xor(sum, 1, 64);
    if constexpr (L >= 4) sum += __shfl_xor(sum, 2, 64);
    if constexpr (L >= 8) sum += __shfl_xor(sum, 4, 64);
    if constexpr (L >= 16) sum += __shfl_xor(sum, 8, 64);
    const int row = c * (64 / L) + lane / L;
    if ((lane & (L - 1)) == 0 && row < N) u[row] = scale ? sum * scale[row] : sum;
  }
}

template <typename T, int L>
static void rows_launch(const RowPlan& rp, const T* v, T* u, const double* scale, const int* done,
                        hipStream_t s, const StageArgs& st) {
  k_rows<T, L><<<rp.nblk, kSliceBlock, 0, s>>>(rp.nlayer, rp.N, rp.layer, rp.hidx, rp.cidx, v, rp.F, u, scale,
                                               done, st);
}

template <typename T>
static void rows_dispatch(const RowPlan& rp, const T* v, T* u, const double* scale, const int* done,
                          hipStream_t s, const StageArgs& st) {
  switch (rp.L) {
    case 1: rows_launch<T, 1>(rp, v, u, scale, done, s, st); break;
    case 2: rows_launch<T, 2>(rp, v, u, scale, done, s, st); break;
    case 4: rows_launch<T, 4>(rp, v, u, scale, done, s, st); break;
    case 8: rows_launch<T, 8>(rp, v, u, scale, done, s, st); break;
    default: rows_launch<T, 16>(rp, v, u, scale, done, s, st); break;
  }
}

template <int L>
static void rows_val_launch(const RowPlan& rp, const double* v, double* u, const double* scale,
                            const int* done, hipStream_t s, const StageArgs& st) {
  k_rows_val<L><<<rp.nblk, kSliceBlock, 0, s>>>(rp.nlayer, rp.N, rp.layer, rp.hidx, rp.hval, rp.cidx, rp.cval,
                                                v, rp.F, u, scale, done, st);
}

static void rows_val_dispatch(const RowPlan& rp, const double* v, double* u, const double* scale,
                              const int* done, hipStream_t s, const StageArgs& st) {
  switch (rp.L) {
    case 1: rows_val_launch<1>(rp, v, u, scale, done, s, st); break;
    case 2: rows_val_launch<2>(rp, v, u, scale, done, s, st); break;
    case 4: rows_val_launch<4>(rp, v, u, scale, done, s, st); break;
    case 8: rows_val_launch<8>(rp, v, u, scale, done, s, st); break;
    default: rows_val_launch<16>(rp, v, u, scale, done, s, st); break;
  }
}

void launch_rows(const RowPlan& rp, const double* v, double* u, const double* scale, const int* done,
                 hipStream_t s, const StageArgs* stage) {
  StageArgs st{};
  if (stage) st = *stage;
  if (rp.nblk > 0 && rp.hval)
    rows_val_dispatch(rp, v, u, scale, done, s, st);
  else if (rp.nblk > 0)
    rows_dispatch<double>(rp, v, u, scale, done, s, st);
  else if (stage)
    launch_stage_update(*stage, s);
}

template <int L>
static void rows_pu_launch(const RowPlan& rp, const double* z, double* up, const double* scale, const int* done,
                           hipStream_t s, const PUpd& pu) {
  k_rows<double, L, true><<<rp.nblk, kSliceBlock, 0, s>>>(rp.nlayer, rp.N, rp.layer, rp.hidx, rp.cidx, z, rp.F,
                                                          up, scale, done, StageArgs{}, pu);
}

void launch_rows_pupd(const RowPlan& rp, const double* z, double* up, const double* scale, const int* done,
                      hipStream_t s, const PUpd& pu) {
  switch (rp.L) {
    case 1: rows_pu_launch<1>(rp, z, up, scale, done, s, pu); break;
    case 2: rows_pu_launch<2>(rp, z, up, scale, done, s, pu); break;
    case 4: rows_pu_launch<4>(rp, z, up, scale, done, s, pu); break;
    case 8: rows_pu_launch<8>(rp, z, up, scale, done, s, pu); break;
    default: rows_pu_launch<16>(rp, z, up, scale, done, s, pu); break;
  }
}

void launch_rows32(const RowPlan& rp, const float* v, float* u, const int* done, hipStream_t s,
                   const StageArgs* stage) {
  StageArgs st{};
  if (stage) st = *stage;
  if (rp.nblk > 0)
    rows_dispatch<float>(rp, v, u, nullptr, done, s, st);
  else if (stage)
    launch_stage_update(*stage, s);
}

void free_rows(RowPlan& rp) {
  if (rp.layer) (void)dev_free(rp.layer);
  if (rp.hidx) (void)dev_free(rp.hidx);
  if (rp.cidx) (void)dev_free(rp.cidx);
  if (rp.hval) (void)dev_free(rp.hval);
  if (rp.cval) (void)dev_free(rp.cval);
  rp = RowPlan{};
}

// Host-side construction from the CSR (columns sorted inside every row, in
// the popularity order).  Setup only.
rr_status build_rows(RowPlan& out, const std::vector<int>& ptr, const std::vector<int>& col, int N, int F,
                     int num_cu, int L, hipStream_t s, const std::vector<double>* val) {
  free_rows(out);
  if (L != 1 && L != 2 && L != 4 && L != 8 && L != 16)
    return fail(RR_ERR_DEVICE, "internal: lanes per row must be 1, 2, 4, 8 or 16");
  const int W = kSliceRows;
  const int rpl = 64 / L;
  const int nlayer = cdiv(N, rpl);
  std::vector<int4> lay(std::max(1, nlayer));
  std::vector<uint16_t> hidx;
  std::vector<int> cidx;
  std::vector<double> hv, cv;   // valued X: values at the indexes' positions
  long long hot = 0, cold = 0;
  std::vector<int> hc(64), cc(64);
  for (int c = 0; c < nlayer; ++c) {
    int hm = 0, cm = 0;
    for (int l = 0; l < 64; ++l) {
      const int i = c * rpl + l / L, sub = l % L;
      hc[l] = cc[l] = 0;
      if (i >= N) continue;
      int h = 0, k2 = 0;
      for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        if (col[k] < W) {
          if (h % L == sub) ++hc[l];
          ++h;
        } else {
          if (k2 % L == sub) ++cc[l];
          ++k2;
        }
      }
      hm = std::max(hm, hc[l]);
      cm = std::max(cm, cc[l]);
    }
    hm = (hm + 3) / 4 * 4;
    cm = (cm + 3) / 4 * 4;
    const size_t hoff = hidx.size(), coff = cidx.size();
    if (hoff + (size_t)hm * 64 > (size_t)INT_MAX || coff + (size_t)cm * 64 > (size_t)INT_MAX)
      return fail(RR_ERR_UNSUPPORTED, "row pass: more than 2^31 padded entries");
    lay[c] = make_int4((int)hoff, hm, (int)coff, cm);
    hidx.resize(hoff + (size_t)hm * 64, (uint16_t)W);
    cidx.resize(coff + (size_t)cm * 64, -1);
    if (val) {
      hv.resize(hidx.size(), 0.0);
      cv.resize(cidx.size(), 0.0);
    }
    for (int l = 0; l < 64; ++l) {
      const int i = c * rpl + l / L, sub = l % L;
      if (i >= N) continue;
      int h = 0, k2 = 0, hs = 0, cs = 0;
      for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int j = col[k];
        if (j < W) {
          if (h % L == sub) {
            const size_t at = hoff + (size_t)(hs / 4) * 256 + 4 * l + hs % 4;
            hidx[at] = (uint16_t)j;
            if (val) hv[at] = (*val)[k];
            ++hs;
          }
          ++h;
        } else {
          if (k2 % L == sub) {
            const size_t at = coff + (size_t)(cs / 4) * 256 + 4 * l + cs % 4;
            cidx[at] = j;
            if (val) cv[at] = (*val)[k];
            ++cs;
          }
          ++k2;
        }
      }
      hot += hs;
      cold += cs;
    }
  }
  // the kernel trusts the plan: check every access it will make
  for (int c = 0; c < nlayer; ++c) {
    const int4 d = lay[c];
    if (d.x % 256 || d.z % 256 || d.y % 4 || d.w % 4 || (size_t)d.x + (size_t)d.y * 64 > hidx.size() ||
        (size_t)d.z + (size_t)d.w * 64 > cidx.size())
      return fail(RR_ERR_DEVICE, "internal: row plan out of range");
  }
  for (uint16_t q : hidx)
    if (q > W) return fail(RR_ERR_DEVICE, "internal: row plan hot index out of range");
  for (int q : cidx)
    if (q != -1 && (q < W || q >= F)) return fail(RR_ERR_DEVICE, "internal: row plan cold index out of range");
  if (hidx.empty()) hidx.resize(256, (uint16_t)W);
  if (cidx.empty()) cidx.resize(256, -1);
  if (val) {
    hv.resize(hidx.size(), 0.0);
    cv.resize(cidx.size(), 0.0);
  }
  out.N = N;
  out.F = F;
  out.W = W;
  out.L = L;
  out.nlayer = nlayer;
  out.nblk = nlayer > 0 ? std::min(std::max(1, num_cu), cdiv(nlayer, kSliceWaves)) : 0;
  out.hot_entries = hot;
  out.cold_entries = cold;
  out.idx_bytes = (long long)hidx.size() * 2 + (long long)cidx.size() * 4;
  RR_HIP(dmalloc(&out.layer, sizeof(int4) * lay.size()));
  RR_HIP(dmalloc(&out.hidx, sizeof(uint16_t) * hidx.size()));
  RR_HIP(dmalloc(&out.cidx, sizeof(int) * cidx.size()));
  RR_HIP(hipMemcpyAsync(out.layer, lay.data(), sizeof(int4) * lay.size(), hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(out.hidx, hidx.data(), sizeof(uint16_t) * hidx.size(), hipMemcpyHostToDevice, s));
  RR_HIP(hipMemcpyAsync(out.cidx, cidx.data(), sizeof(int) * cidx.size(), hipMemcpyHostToDevice, s));
  if (val) {
    RR_HIP(dmalloc(&out.hval, sizeof(double) * hv.size()));
    RR_HIP(dmalloc(&out.cval, sizeof(double) * cv.size()));
    RR_HIP(hipMemcpyAsync(out.hval, hv.data(), sizeof(double) * hv.size(), hipMemcpyHostToDevice, s));
    RR_HIP(hipMemcpyAsync(out.cval, cv.data(), sizeof(double) * cv.size(), hipMemcpyHostToDevice, s));
    out.idx_bytes += (long long)(hv.size() + cv.size()) * 8;
  }
  RR_HIP(hipStreamSynchronize(s));
  return RR_OK;
}

}  // namespace rr
