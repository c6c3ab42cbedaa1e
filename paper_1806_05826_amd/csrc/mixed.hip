// Single-precision vector kernels of the inner solves of iterative
// refinement: the correction equation A d = r is solved by PCG with FP32
// vectors and FP32 operator sums, while the scalars (alpha, beta, norms) are
// formed and kept in FP64 and the coarse solve stays FP64.  The outer
// residual r = b - A x is recomputed in FP64 after each inner solve.
#include "rr_device.h"

namespace rr {

// Inner start: r32 = r (rounded), d = 0, p = 0, D32 = c + lambda, and the
// first smoother step; partials of ||r32||^2 and <r32, z> (Jacobi) in FP64.
__global__ __launch_bounds__(kBlock) void k_ir_init(int F, const double* __restrict__ r64,
                                                    const double* __restrict__ colnorm,
                                                    double lam, double omega, int kind,
                                                    IrVectors v, double* parts) {
  double b0 = 0.0, b2 = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const float rj = (float)r64[j];
    const float Dj = (float)(colnorm[j] + lam);
    v.r[j] = rj;
    v.x[j] = 0.0f;
    v.p[j] = 0.0f;
    v.D[j] = Dj;
    b0 += (double)rj * (double)rj;
    if (kind == PK_JACOBI) {
      const float zj = rj / Dj;
      v.z[j] = zj;
      b2 += (double)rj * (double)zj;
    } else if (kind == PK_NONE) {
      v.z[j] = rj;
      b2 += (double)rj * (double)rj;
    } else {
      v.e1[j] = ((float)omega * rj) / Dj;
    }
  }
  __shared__ double red[kBlock / 64];
  const double t0 = block_sum(b0, red);
  const double t2 = block_sum(b2, red);
  if (threadIdx.x == 0) {
    parts[blockIdx.x] = t0;
    parts[gridDim.x + blockIdx.x] = 0.0;
    parts[2 * gridDim.x + blockIdx.x] = t2;
  }
}

// The FP32 cycle of an FP64 flexible-CG solve: r32 = (float) r, D32, and
// the pre-smoothing step e1 = w D^-1 r in FP32 (skipped once the solve is done).
__global__ __launch_bounds__(kBlock) void k_cycle_in(int F, const double* __restrict__ r64,
                                                     const double* __restrict__ colnorm, double lam,
                                                     double omega, IrVectors v, const int* done) {
  if (is_done(done)) return;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const float rj = (float)r64[j];
    const float Dj = (float)(colnorm[j] + lam);
    v.r[j] = rj;
    v.D[j] = Dj;
    v.e1[j] = ((float)omega * rj) / Dj;
  }
}
void launch_cycle_in(int F, const double* r64, const double* colnorm, double lam, double omega,
                     const IrVectors& v, const int* done, hipStream_t s) {
  k_cycle_in<<<vec_grid(F), kBlock, 0, s>>>(F, r64, colnorm, lam, omega, v, done);
}

// z = (double) z32
__global__ __launch_bounds__(kBlock) void k_widen(int F, const float* __restrict__ z32,
                                                  double* __restrict__ z, const int* done) {
  if (is_done(done)) return;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) z[j] = (double)z32[j];
}
void launch_widen(int F, const float* z32, double* z, const int* done, hipStream_t s) {
  k_widen<<<vec_grid(F), kBlock, 0, s>>>(F, z32, z, done);
}

void launch_ir_init(int F, const double* r64, const double* colnorm, double lam, double omega,
                    int kind, const IrVectors& v, double* parts, hipStream_t s) {
  k_ir_init<<<vec_grid(F), kBlock, 0, s>>>(F, r64, colnorm, lam, omega, kind, v, parts);
}

// alpha = <r,z> / <p,Ap> in FP64; d += alpha p; r -= alpha q (FP32); the next
// smoother input; FP64 partials of ||r||^2 and <r,z> (Jacobi / CG forms).
__global__ __launch_bounds__(kBlock) void k_ir_update(int F, IrVectors v, double omega, int kind,
                                                      Scalars* sc, const double* parts_pq,
                                                      int n_pq, double* parts_upd) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  const double pq = sum_parts<kBlock>(parts_pq, n_pq, red);
  if (!finite_pos(pq)) {
    if (is_block0_lead()) {
      sc->pq = pq;
      sc->status = RR_ERR_BREAKDOWN;
      sc->done = 1;
    }
    return;
  }
  const double rz = sc->rz_next;
  const double alpha = rz / pq;
  if (is_block0_lead()) {
    sc->pq = pq;
    sc->alpha = alpha;
    sc->rz = rz;
    sc->iter = sc->iter + 1;
  }
  const float a = (float)alpha;
  const float w = (float)omega;
  double v0 = 0.0, v2 = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    v.x[j] += a * v.p[j];
    const float rj = v.r[j] - a * v.q[j];
    v.r[j] = rj;
    v0 += (double)rj * (double)rj;
    if (kind == PK_JACOBI) {
      const float zj = rj / v.D[j];
      v.z[j] = zj;
      v2 += (double)rj * (double)zj;
    } else if (kind == PK_NONE) {
      v.z[j] = rj;
      v2 += (double)rj * (double)rj;
    } else {
      v.e1[j] = (w * rj) / v.D[j];
    }
  }
  const double t0 = block_sum(v0, red);
  const double t2 = block_sum(v2, red);
  if (threadIdx.x == 0) {
    parts_upd[blockIdx.x] = t0;
    parts_upd[gridDim.x + blockIdx.x] = 0.0;
    parts_upd[2 * gridDim.x + blockIdx.x] = t2;
  }
}

void launch_ir_update(int F, const IrVectors& v, double omega, int kind, Scalars* sc,
                      const double* parts_pq, int n_pq, double* parts_upd, hipStream_t s) {
  k_ir_update<<<vec_grid(F), kBlock, 0, s>>>(F, v, omega, kind, sc, parts_pq, n_pq, parts_upd);
}

// p = z + beta p (FP32) with beta from FP64 <r,z>; first: beta = 0.  With a
// stage, the convergence check of the preceding update runs first.
__global__ __launch_bounds__(kBlock) void k_ir_pupdate(int F, float* __restrict__ p,
                                                       const float* __restrict__ z, Scalars* sc,
                                                       const double* __restrict__ parts_rz,
                                                       int n_rz, int first, StageArgs stage) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  double rz_new;
  if (stage.sc) {
    if (stage_update<kBlock>(stage, red, rz_new)) return;
  } else {
    rz_new = sum_parts<kBlock>(parts_rz, n_rz, red);
  }
  if (!finite_pos(rz_new)) {
    if (is_block0_lead()) {
      sc->status = RR_ERR_BREAKDOWN;
      sc->done = 1;
    }
    return;
  }
  const double beta = first ? 0.0 : rz_new / sc->rz;
  if (is_block0_lead()) {
    sc->rz_next = rz_new;
    sc->beta = beta;
  }
  const float b = (float)beta;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock)
    p[j] = z[j] + b * p[j];
}

void launch_ir_pupdate(int F, float* p, const float* z, Scalars* sc, const double* parts_rz,
                       int n_rz, int first, const StageArgs* stage, hipStream_t s) {
  StageArgs st{};
  if (stage) st = *stage;
  k_ir_pupdate<<<vec_grid(F), kBlock, 0, s>>>(F, p, z, sc, parts_rz, n_rz, first, st);
}

// e2 = e1 + P yc (rounded to FP32).
__global__ __launch_bounds__(kBlock) void k_prolong32(int F, const int* __restrict__ labels,
                                                      const double* __restrict__ cscale,
                                                      const double* __restrict__ yc,
                                                      const float* __restrict__ e1,
                                                      float* __restrict__ e2, const int* done) {
  if (is_done(done)) return;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const int s = labels[j];
    e2[j] = e1[j] + (float)(cscale[s] * yc[s]);
  }
}

void launch_prolong32(int F, const int* labels, const double* cscale, const double* yc,
                      const float* e1, float* e2, const int* done, hipStream_t s) {
  k_prolong32<<<vec_grid(F), kBlock, 0, s>>>(F, labels, cscale, yc, e1, e2, done);
}

// x += d (FP64 accumulation of the FP32 correction).
__global__ void k_ir_accumulate(int F, double* __restrict__ x, const float* __restrict__ d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) x[j] += (double)d[j];
}

void launch_ir_accumulate(int F, double* x, const float* d, hipStream_t s) {
  k_ir_accumulate<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, x, d);
}

}  // namespace rr
