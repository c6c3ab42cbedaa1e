// Device helpers shared by the HIP kernels: block reductions and the
// last-block ticket that finishes a grid-wide reduction in a fixed order.
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

// Block-reduce NV values and store them in partial slot `slot` of
// `partials` (layout partials[i * nslots + slot]).
template <int NV>
__device__ inline void write_partial(const double (&v)[NV], double* partials, int slot,
                                     int nslots) {
  __shared__ double red[kBlock / 64];
  double bs[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) bs[i] = block_sum(v[i], red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i)
      __hip_atomic_store(&partials[i * nslots + slot], bs[i], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Wait until this thread's earlier memory operations have completed.  The
// partials below are written with agent-scope (coherent) atomic stores, so
// once they have completed every block can see them; no cache writeback of
// the whole L2 is needed, unlike a full release fence.
__device__ inline void wait_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Every block of the grid stores its partial in slot (slot0 + blockIdx.x);
// the last block to arrive then adds all `nslots` partials (which may include
// slots written by an earlier kernel) in slot order, and returns true with
// the totals in `tot` (valid in every thread of that block).  Partials are
// agent-scope atomic stores and loads; the arrival ticket is an agent-scope
// atomic counter, reset by the last block.
template <int NV>
__device__ inline bool grid_finish(const double (&v)[NV], double* partials, int slot0,
                                   int nslots, unsigned int* ticket, double (&tot)[NV]) {
  __shared__ double red2[kBlock / 64];
  __shared__ int is_last;
  write_partial<NV>(v, partials, slot0 + blockIdx.x, nslots);
  if (threadIdx.x == 0) {
    wait_stores();
    const unsigned int prev =
        __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == (unsigned)gridDim.x - 1u);
  }
  __syncthreads();
  if (!is_last) return false;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int j = threadIdx.x; j < nslots; j += kBlock)
      s += __hip_atomic_load(&partials[i * nslots + j], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    tot[i] = block_sum(s, red2);
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

__device__ inline bool finite_pos(double v) { return v > 0.0 && v < __builtin_inf(); }

// Scalar updates done by the finishing block (thread 0 only).
__device__ inline void finish_alpha(Scalars* sc, double pq) {
  sc->pq = pq;
  if (!finite_pos(pq)) {
    sc->status = RR_ERR_BREAKDOWN;
    sc->done = 1;
  } else {
    sc->alpha = sc->rz / pq;
  }
}

__device__ inline void finish_beta(Scalars* sc, double rz_new) {
  if (!finite_pos(rz_new)) {
    sc->status = RR_ERR_BREAKDOWN;
    sc->done = 1;
    return;
  }
  sc->beta = (sc->iter == 0) ? 0.0 : rz_new / sc->rz;
  sc->rz = rz_new;
}

__device__ inline bool is_done(const int* done) { return done != nullptr && *done != 0; }

}  // namespace rr
