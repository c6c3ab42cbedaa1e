// Device helpers shared by the HIP kernels: block reductions, the sums of
// block partials that every consumer block repeats in the same order, the
// solver's convergence check, and the column epilogues.
#pragma once

#include "rr_internal.h"

namespace rr {

// Sum of v over the block (kBlock threads); result valid in every thread.
// The tree is fixed, so the result is deterministic.
__device__ inline double block_sum(double v, double* lds /* kBlock/64 */) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) t += lds[i];
  __syncthreads();
  return t;
}

// Sum over a block of NT threads; result in every thread; fixed tree.
template <int NT>
__device__ inline double block_sum_n(double v, double* lds /* NT/64 */) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += lds[i];
  __syncthreads();
  return t;
}

// Every block calls this with the same (p, n) and gets the same total: the
// partials of a previous kernel added in one fixed order.
template <int NT>
__device__ inline double sum_parts(const double* p, int n, double* lds) {
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) s += p[j];
  return block_sum_n<NT>(s, lds);
}

// Wait until this thread's earlier memory operations have completed.  Used
// after agent-scope (coherent) atomic stores that another block will read
// once it has seen a later ticket; no cache writeback of the whole L2 is
// needed, unlike a full release fence.
__device__ inline void wait_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ inline bool finite_pos(double v) { return v > 0.0 && v < __builtin_inf(); }

__device__ inline bool is_done(const int* done) { return done != nullptr && *done != 0; }

__device__ inline bool is_block0_lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

// The convergence check after an x/r update, run by every block of the
// kernel that follows the update (all blocks reach the same decision from
// the same partials; block 0 records it).  The update kernel has already
// advanced the iteration count.  Returns true when the solve is finished;
// rz_new receives <r,z> of the new residual (Jacobi / CG forms).
template <int NT>
__device__ inline bool stage_update(const StageArgs& st, double* lds, double& rz_new) {
  Scalars* sc = st.sc;
  const double rr = sum_parts<NT>(st.upd, st.n, lds);
  const double ee = sum_parts<NT>(st.upd + st.n, st.n, lds);
  rz_new = sum_parts<NT>(st.upd + 2 * st.n, st.n, lds);
  const int it = sc->iter;
  bool fin = false;
  int status = RR_ERR_NOT_CONVERGED;
  if (!(rr == rr)) {
    fin = true;
    status = RR_ERR_BREAKDOWN;
  } else if (sc->fixed > 0) {
    if (it >= sc->fixed) {
      fin = true;
      status = RR_OK;
    }
  } else if (rr <= sc->tol2 || (sc->use_err && ee <= sc->errtol2)) {
    fin = true;
    status = RR_OK;
  } else if (it >= sc->limit) {
    fin = true;
  }
  if (is_block0_lead()) {
    sc->rr = rr;
    sc->ee = ee;
    if (st.history) st.history[it] = sqrt(rr / sc->bb);
    if (fin) {
      sc->status = status;
      sc->done = 1;
    }
  }
  return fin;
}

// dst[0, W] = src[0, n) followed by zeros (n <= W = kSliceRows), with direct
// global-to-LDS loads: at step k wave w moves the 64 E entries starting at
// (16 k + w) 64 E, 16 bytes (E entries) per lane; the entries past the last
// whole E-group below n and the zero tail are written one by one.  The
// caller waits for the loads (s_waitcnt) and synchronises the workgroup.
template <typename T>
__device__ inline void fill_slice(T* dst, const T* __restrict__ src, int n) {
  constexpr int E = 16 / (int)sizeof(T);
  constexpr int ROW = 64 * E;
  static_assert(kSliceRows % (kSliceWaves * ROW) == 0, "slice copy covers whole 1 KB rows");
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nfull = n - n % E;
#pragma unroll
  for (int k = 0; k < kSliceRows / (kSliceWaves * ROW); ++k) {
    const int e0 = (k * kSliceWaves + w) * ROW;
    if (e0 + E * lane < nfull)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(src + e0 + E * lane),
          (__attribute__((address_space(3))) void*)(dst + e0), 16, 0, 0);
  }
  for (int i = nfull + (int)threadIdx.x; i <= kSliceRows; i += kSliceBlock)
    dst[i] = (i < n) ? src[i] : T(0);
}

// Segment epilogues: what happens to a finished column sum t of column s.
template <int MODE>
__device__ inline void seg_finish(int s, double t, const Epi& e, double& dot) {
  if constexpr (MODE == EPI_STORE) {
    e.out[s] = t;
  } else if constexpr (MODE == EPI_APPLY) {
    e.out[s] = t + e.lam * e.p[s];
  } else if constexpr (MODE == EPI_APPLY_DOT) {
    const double ps = e.p[s];
    const double q = t + e.lam * ps;
    e.out[s] = q;
    dot += ps * q;
  } else if constexpr (MODE == EPI_APPLY_DOT_P) {
    const double ps = e.r[s] + e.sc->beta * e.p[s];
    e.pnew[s] = ps;
    const double q = t + e.lam * ps;
    e.out[s] = q;
    dot += ps * q;
  } else if constexpr (MODE == EPI_RESID) {
    e.out[e.opos ? e.opos[s] : s] = e.r[s] - (t + e.lam * e.p[s]);
  } else if constexpr (MODE == EPI_POST) {
    const double e2 = e.p[s];
    const double rs = e.r[s];
    const double rho = rs - (t + e.lam * e2);
    const double z = e2 + (e.omega * rho) / e.D[s];
    e.out[s] = z;
    dot += rs * z;
  } else if constexpr (MODE == EPI_POST_P) {
    const int l = e.labels[s];
    const double e2 = e.p[s] + e.cscale[l] * e.yc[l];
    const double rs = e.r[s];
    const double rho = rs - (t + e.lam * e2);
    const double z = e2 + (e.omega * rho) / e.D[s];
    e.out[s] = z;
    dot += rs * z;
  } else if constexpr (MODE == EPI_TRUE) {
    const double res = e.r[s] - (t + e.lam * e.p[s]);
    if (e.out) e.out[s] = res;
    dot += res * res;
  } else if constexpr (MODE == EPI_SCALE) {
    e.out[s] = t * e.scale[s];
  }
}

template <int MODE>
constexpr bool has_dot() {
  return MODE == EPI_APPLY_DOT || MODE == EPI_APPLY_DOT_P || MODE == EPI_POST || MODE == EPI_POST_P ||
         MODE == EPI_TRUE;
}

// The epilogue's dot product leaves one partial per block (consumed by the
// next solver kernel).
template <int NT>
__device__ inline void store_block_partial(double v, double* partials, int slot) {
  __shared__ double red_p[NT / 64];
  const double t = block_sum_n<NT>(v, red_p);
  if (threadIdx.x == 0) partials[slot] = t;
}
}  // namespace rr
