// Fused vector kernels of the PCG iteration (the x/r updates and the
// scalars of the flexible-CG algorithm's update steps, specialised to a
// fixed preconditioner).  A reduction leaves one partial per block; every
// block of the kernel that needs the scalar adds the partials itself in slot
// order, so scalars stay on the device, no block waits for another, and
// results are bitwise reproducible run to run.
#include "rr_device.h"

namespace rr {

int vec_grid(int F) { return std::max(1, std::min(kMaxParts, cdiv(F, kBlock))); }

// Block partials of up to three sums, stored in parts[i * n + blockIdx.x].
__device__ inline void store_parts3(double a, double b, double c, double* parts, int n) {
  __shared__ double red[kBlock / 64];
  const double ta = block_sum(a, red);
  const double tb = block_sum(b, red);
  const double tc = block_sum(c, red);
  if (threadIdx.x == 0) {
    parts[blockIdx.x] = ta;
    parts[n + blockIdx.x] = tb;
    parts[2 * n + blockIdx.x] = tc;
  }
}

// x = 0, r = b, p = 0, the first smoother step, and the partials of ||b||^2,
// ||x_ref||^2 and <r, z> (Jacobi / CG forms).
__global__ __launch_bounds__(kBlock) void k_pcg_init(int F, const double* __restrict__ b,
                                                     double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     double* __restrict__ p,
                                                     double* __restrict__ z,
                                                     double* __restrict__ e1,
                                                     const double* __restrict__ D,
                                                     const double* __restrict__ xref,
                                                     double omega, int kind, double* parts) {
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const double bj = b[j];
    x[j] = 0.0;
    r[j] = bj;
    p[j] = 0.0;
    v0 += bj * bj;
    if (xref) v1 += xref[j] * xref[j];
    if (kind == PK_JACOBI) {
      const double zj = bj / D[j];
      z[j] = zj;
      v2 += bj * zj;
    } else if (kind == PK_NONE) {
      z[j] = bj;
      v2 += bj * bj;
    } else if (kind == PK_VCYCLE || kind == PK_LEARNED) {
      e1[j] = (omega * bj) / D[j];
    }
  }
  store_parts3(v0, v1, v2, parts, gridDim.x);
}

void launch_pcg_init(int F, const double* b, double* x, double* r, double* p, double* z,
                     double* e1, const double* D, const double* xref, double omega, int kind,
                     double* parts_init, hipStream_t s) {
  k_pcg_init<<<vec_grid(F), kBlock, 0, s>>>(F, b, x, r, p, z, e1, D, xref, omega, kind,
                                            parts_init);
}

// ||b||^2 and ||x_ref||^2 from the init partials; scales the tolerances.
__global__ __launch_bounds__(kBlock) void k_finish_init(Scalars* sc, const double* parts, int n,
                                                        double* history) {
  __shared__ double red[kBlock / 64];
  const double bb = sum_parts<kBlock>(parts, n, red);
  const double ref2 = sum_parts<kBlock>(parts + n, n, red);
  if (threadIdx.x != 0) return;
  sc->bb = bb;
  sc->ref2 = ref2;
  sc->tol2 *= bb;
  sc->errtol2 *= ref2;
  sc->iter = 0;
  if (history) history[0] = (bb > 0.0) ? 1.0 : 0.0;
  if (!(bb > 0.0)) {
    sc->done = 1;
    sc->status = (bb == 0.0) ? RR_OK : RR_ERR_BREAKDOWN;
    sc->true_rr = 0.0;
  }
}

void launch_finish_init(Scalars* sc, const double* parts_init, int n, double* history, int,
                        hipStream_t s) {
  k_finish_init<<<1, kBlock, 0, s>>>(sc, parts_init, n, history);
}

// alpha = <r,z> / <p,Ap> (every block adds the <p,Ap> partials itself), then
// x += alpha p; r -= alpha q; the next smoother input; partials of ||r||^2,
// the error and <r, z> (Jacobi / CG forms).  The convergence check runs in
// the next kernel.
__global__ __launch_bounds__(kBlock) void k_pcg_update(
    int F, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ z, double* __restrict__ e1,
    const double* __restrict__ D, const double* __restrict__ xref, double omega, int kind,
    Scalars* sc, const double* __restrict__ parts_pq, int n_pq, double* parts_upd) {
  // this thread's first entry is loaded before the done flag and the
  // partials, so that the three loads are in flight together
  const int j0 = blockIdx.x * kBlock + threadIdx.x;
  const bool need_d = kind == PK_JACOBI || kind == PK_VCYCLE || kind == PK_LEARNED;
  double x0 = 0.0, p0 = 0.0, r0 = 0.0, q0 = 0.0, d0 = 1.0, xr0 = 0.0;
  if (j0 < F) {
    x0 = x[j0];
    p0 = p[j0];
    r0 = r[j0];
    q0 = q[j0];
    if (need_d) d0 = D[j0];
    if (xref) xr0 = xref[j0];
  }
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
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  auto entry = [&](int j, double xo, double pj, double ro, double qj, double dj, double xrj) {
    const double xj = xo + alpha * pj;
    const double rj = ro - alpha * qj;
    x[j] = xj;
    r[j] = rj;
    v0 += rj * rj;
    if (xref) {
      const double d = xj - xrj;
      v1 += d * d;
    }
    if (kind == PK_JACOBI) {
      const double zj = rj / dj;
      z[j] = zj;
      v2 += rj * zj;
    } else if (kind == PK_NONE) {
      z[j] = rj;
      v2 += rj * rj;
    } else if (kind == PK_VCYCLE || kind == PK_LEARNED) {
      e1[j] = (omega * rj) / dj;
    }
  };
  if (j0 < F) entry(j0, x0, p0, r0, q0, d0, xr0);
  for (int j = j0 + gridDim.x * kBlock; j < F; j += gridDim.x * kBlock)
    entry(j, x[j], p[j], r[j], q[j], need_d ? D[j] : 1.0, xref ? xref[j] : 0.0);
  store_parts3(v0, v1, v2, parts_upd, gridDim.x);
}

void launch_pcg_update(int F, double* x, double* r, const double* p, const double* q,
                       double* z, double* e1, const double* D, const double* xref,
                       double omega, int kind, Scalars* sc, const double* parts_pq, int n_pq,
                       double* parts_upd, hipStream_t s) {
  k_pcg_update<<<vec_grid(F), kBlock, 0, s>>>(F, x, r, p, q, z, e1, D, xref, omega, kind, sc,
                                              parts_pq, n_pq, parts_upd);
}

// p = z + beta p with beta = <r,z>_new / <r,z>_old (0 on the first call).
// With a stage, the convergence check of the preceding update runs first and
// <r,z> comes from the update's partials.
__global__ __launch_bounds__(kBlock) void k_pupdate(int F, double* __restrict__ p,
                                                    const double* __restrict__ z, Scalars* sc,
                                                    const double* __restrict__ parts_rz,
                                                    int n_rz, int first, StageArgs stage) {
  const int j0 = blockIdx.x * kBlock + threadIdx.x;
  double z0 = 0.0, p0 = 0.0;   // loaded together with the done flag and the partials
  if (j0 < F) {
    z0 = z[j0];
    p0 = p[j0];
  }
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
  if (j0 < F) p[j0] = z0 + beta * p0;
  for (int j = j0 + gridDim.x * kBlock; j < F; j += gridDim.x * kBlock) p[j] = z[j] + beta * p[j];
}

void launch_pupdate(int F, double* p, const double* z, Scalars* sc, const double* parts_rz,
                    int n_rz, int first, const StageArgs* stage, hipStream_t s) {
  StageArgs st{};
  if (stage) st = *stage;
  k_pupdate<<<vec_grid(F), kBlock, 0, s>>>(F, p, z, sc, parts_rz, n_rz, first, st);
}

// The convergence check alone (one block), where the next kernel cannot
// host it.
__global__ __launch_bounds__(kBlock) void k_stage_update(StageArgs st) {
  if (st.sc->done) return;
  __shared__ double red[kBlock / 64];
  double rz_unused;
  (void)stage_update<kBlock>(st, red, rz_unused);
}

void launch_stage_update(const StageArgs& st, hipStream_t s) {
  k_stage_update<<<1, kBlock, 0, s>>>(st);
}

// ||b - A x||^2 from the partials of the true-residual pass.
__global__ __launch_bounds__(kBlock) void k_finish_true(Scalars* sc, const double* parts, int n) {
  __shared__ double red[kBlock / 64];
  const double t = sum_parts<kBlock>(parts, n, red);
  if (threadIdx.x == 0) sc->true_rr = t;
}

void launch_finish_true(Scalars* sc, const double* parts, int n, hipStream_t s) {
  k_finish_true<<<1, kBlock, 0, s>>>(sc, parts, n);
}

// Prolongation: out = e1 + P yc (V-cycle), or the additive form
// z = w D^-1 r + P yc with partials of <r,z>.  P(j, s) is cscale[s] (adjusted
// square-root average) or, with pw, the feature's own weight pw[j]
// (least-squares interpolation).
__global__ __launch_bounds__(kBlock) void k_prolong(int F, const int* __restrict__ labels,
                                                    const double* __restrict__ cscale,
                                                    const double* __restrict__ pw,
                                                    const double* __restrict__ yc,
                                                    const double* __restrict__ e1,
                                                    double* __restrict__ out,
                                                    const double* __restrict__ r,
                                                    const double* __restrict__ D, double omega,
                                                    int additive, const Scalars* sc,
                                                    double* parts_rz) {
  // this thread's first label and operands are loaded before the done flag
  const int j0 = blockIdx.x * kBlock + threadIdx.x;
  int l0 = 0;
  double a0 = 0.0, d0 = 1.0;
  if (j0 < F) {
    l0 = labels[j0];
    a0 = additive ? r[j0] : e1[j0];
    if (additive) d0 = D[j0];
  }
  if (sc && sc->done) return;
  double v = 0.0;
  auto entry = [&](int j, int s, double a, double dj) {
    const double corr = (pw ? pw[j] : cscale[s]) * yc[s];
    if (additive) {
      const double zj = (omega * a) / dj + corr;
      out[j] = zj;
      v += a * zj;
    } else {
      out[j] = a + corr;
    }
  };
  if (j0 < F) entry(j0, l0, a0, d0);
  for (int j = j0 + gridDim.x * kBlock; j < F; j += gridDim.x * kBlock)
    entry(j, labels[j], additive ? r[j] : e1[j], additive ? D[j] : 1.0);
  if (parts_rz) store_block_partial<kBlock>(v, parts_rz, blockIdx.x);
}

void launch_prolong(int F, const int* labels, const double* cscale, const double* yc,
                    const double* e1, double* out, const double* r, const double* D,
                    double omega, int additive, const Scalars* sc, double* parts_rz,
                    hipStream_t s, const double* pw) {
  k_prolong<<<vec_grid(F), kBlock, 0, s>>>(F, labels, cscale, pw, yc, e1, out, r, D, omega,
                                           additive, sc, parts_rz);
}

// ---- flexible CG (truncated, m previous directions) -------------------------

// <z, A p_k> for the window's directions: partials parts[k * gridDim + block].
// With a stage, the convergence check of the preceding update runs first.
__global__ __launch_bounds__(kBlock) void k_fcg_dots(int F, const double* z, FcgWindow win,
                                                     double* parts, Scalars* sc, StageArgs stage) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  if (stage.sc) {
    double rz_unused;
    if (stage_update<kBlock>(stage, red, rz_unused)) return;
  }
  double acc[kMaxFcg];
#pragma unroll
  for (int k = 0; k < kMaxFcg; ++k) acc[k] = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const double zj = z[j];
#pragma unroll
    for (int k = 0; k < kMaxFcg; ++k)
      if (k < win.n) acc[k] += zj * win.ap[k][j];
  }
#pragma unroll
  for (int k = 0; k < kMaxFcg; ++k) {
    if (k < win.n) {
      const double t = block_sum(acc[k], red);
      if (threadIdx.x == 0) parts[k * gridDim.x + blockIdx.x] = t;
    }
  }
}

void launch_fcg_dots(int F, const double* z, const FcgWindow& win, double* parts, Scalars* sc,
                     const StageArgs* stage, hipStream_t s) {
  StageArgs st{};
  if (stage) st = *stage;
  k_fcg_dots<<<vec_grid(F), kBlock, 0, s>>>(F, z, win, parts, sc, st);
}

// p = z - sum_k (<z, A p_k> / <p_k, A p_k>) p_k, oldest direction first, and
// the partials of <p, r>.  p may be the storage of the window's oldest
// direction: each element is read before it is overwritten by the same thread.
__global__ __launch_bounds__(kBlock) void k_fcg_dir(int F, const double* z, const double* r,
                                                    double* p, FcgWindow win,
                                                    const double* dots, int n_dots,
                                                    const double* paps, double* parts_pr,
                                                    const Scalars* sc) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  double c[kMaxFcg];
#pragma unroll
  for (int k = 0; k < kMaxFcg; ++k)
    c[k] = (k < win.n) ? sum_parts<kBlock>(dots + k * n_dots, n_dots, red) / paps[win.slot[k]] : 0.0;
  double v = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    double pj = z[j];
#pragma unroll
    for (int k = 0; k < kMaxFcg; ++k)
      if (k < win.n) pj -= c[k] * win.p[k][j];
    p[j] = pj;
    v += pj * r[j];
  }
  store_block_partial<kBlock>(v, parts_pr, blockIdx.x);
}

void launch_fcg_dir(int F, const double* z, const double* r, double* p, const FcgWindow& win,
                    const double* dots, const double* paps, double* parts_pr, const Scalars* sc,
                    hipStream_t s) {
  k_fcg_dir<<<vec_grid(F), kBlock, 0, s>>>(F, z, r, p, win, dots, vec_grid(F), paps, parts_pr, sc);
}

// alpha = <p, r> / <p, A p>; x += alpha p; r -= alpha q; <p, A p> kept for
// the later orthogonalizations; the next smoother input and the partials of
// ||r||^2 and the error, as in the PCG update.
__global__ __launch_bounds__(kBlock) void k_fcg_update(
    int F, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ z, double* __restrict__ e1,
    const double* __restrict__ D, const double* __restrict__ xref, double omega, int kind,
    Scalars* sc, const double* __restrict__ parts_pq, int n_pq, const double* __restrict__ parts_pr,
    int n_pr, double* paps, int slot, double* parts_upd) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  const double pq = sum_parts<kBlock>(parts_pq, n_pq, red);
  const double pr = sum_parts<kBlock>(parts_pr, n_pr, red);
  if (!finite_pos(pq) || !(pr == pr) || pr == __builtin_inf() || pr == -__builtin_inf()) {
    // under the learned correction the host falls back to the algebraic
    // cycle; x and r keep the last good iterate
    if (is_block0_lead()) {
      sc->pq = pq;
      sc->status = kind == PK_LEARNED ? kStatusFallback : RR_ERR_BREAKDOWN;
      sc->done = 1;
    }
    return;
  }
  const double alpha = pr / pq;
  if (is_block0_lead()) {
    sc->pq = pq;
    sc->alpha = alpha;
    paps[slot] = pq;
    sc->iter = sc->iter + 1;
  }
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const double xj = x[j] + alpha * p[j];
    const double rj = r[j] - alpha * q[j];
    x[j] = xj;
    r[j] = rj;
    v0 += rj * rj;
    if (xref) {
      const double d = xj - xref[j];
      v1 += d * d;
    }
    if (kind == PK_JACOBI) {
      z[j] = rj / D[j];
    } else if (kind == PK_NONE) {
      z[j] = rj;
    } else if (kind == PK_VCYCLE || kind == PK_LEARNED) {
      e1[j] = (omega * rj) / D[j];
    }
  }
  store_parts3(v0, v1, v2, parts_upd, gridDim.x);
}

void launch_fcg_update(int F, double* x, double* r, const double* p, const double* q, double* z,
                       double* e1, const double* D, const double* xref, double omega, int kind,
                       Scalars* sc, const double* parts_pq, int n_pq, const double* parts_pr,
                       double* paps, int slot, double* parts_upd, hipStream_t s) {
  k_fcg_update<<<vec_grid(F), kBlock, 0, s>>>(F, x, r, p, q, z, e1, D, xref, omega, kind, sc,
                                              parts_pq, n_pq, parts_pr, vec_grid(F), paps, slot,
                                              parts_upd);
}

// dst = src unless the solve has finished
__global__ void k_copy_done(double* __restrict__ dst, const double* __restrict__ src, int n,
                            const int* done) {
  if (is_done(done)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
void launch_copy_done(double* dst, const double* src, int n, const int* done, hipStream_t s) {
  if (n > 0) k_copy_done<<<cdiv(n, kBlock), kBlock, 0, s>>>(dst, src, n, done);
}

__global__ void k_fill(double* x, double v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
void launch_fill(double* x, double v, long long n, hipStream_t s) {
  if (n > 0) k_fill<<<cdiv(n, kBlock), kBlock, 0, s>>>(x, v, n);
}

__global__ void k_gather(double* dst, const double* src, const int* idx, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}
void launch_gather(double* dst, const double* src, const int* idx, int n, hipStream_t s) {
  if (n > 0) k_gather<<<cdiv(n, kBlock), kBlock, 0, s>>>(dst, src, idx, n);
}

__global__ void k_copy(double* dst, const double* src, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
void launch_copy(double* dst, const double* src, long long n, hipStream_t s) {
  if (n > 0) k_copy<<<cdiv(n, kBlock), kBlock, 0, s>>>(dst, src, n);
}

__global__ void k_diag(int F, const double* colnorm, double lam, double* D) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) D[j] = colnorm[j] + lam;
}
void launch_colnorm_diag(int F, const double* colnorm, double lam, double* D, hipStream_t s) {
  k_diag<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, colnorm, lam, D);
}

__global__ void k_jacobi(int F, const double* r, const double* D, double* z) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) z[j] = r[j] / D[j];
}
void launch_jacobi_apply(int F, const double* r, const double* D, double* z, hipStream_t s) {
  k_jacobi<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, r, D, z);
}

// rho_hat = max_j (g_j + lam) / (c_j + lam); out = 1 / rho_hat.  One block.
__global__ __launch_bounds__(1024) void k_omega_gersh(int F, const double* g, const double* c,
                                                      double lam, double* out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int j = threadIdx.x; j < F; j += 1024) m = fmax(m, (g[j] + lam) / (c[j] + lam));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = 1.0 / red[0];
}
void launch_omega_gersh(int F, const double* g, const double* colnorm, double lam, double* out,
                        double*, unsigned*, hipStream_t s) {
  k_omega_gersh<<<1, 1024, 0, s>>>(F, g, colnorm, lam, out);
}

// y = A x, A row-major n x n: one wave per row; lane l takes columns
// l + 64 k, 16 loads of A and of x in flight at a time (a whole row when
// n <= 1024, the coarse sizes of interest).
__global__ __launch_bounds__(kBlock) void k_gemv(int n, const double* __restrict__ A,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y, const int* done) {
  if (is_done(done)) return;
  const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* a = A + (size_t)row * n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = lane; c0 < n; c0 += 1024) {
    double av[16], xv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = c0 + 64 * k;
      av[k] = c < n ? a[c] : 0.0;
      xv[k] = c < n ? x[c] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k & 3] += av[k] * xv[k];
  }
  double t = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if (lane == 0) y[row] = t;
}
void launch_gemv(int n, const double* A, const double* x, double* y, const int* done,
                 hipStream_t s) {
  if (n > 0) k_gemv<<<cdiv(n, kBlock / 64), kBlock, 0, s>>>(n, A, x, y, done);
}

// ---- CG rougher: CG on A e = r from e = 0 (plain, or Jacobi-preconditioned when D
// is given; then the partials are <r, D^-1 r> and the directions D^-1 r + beta p) --

__global__ __launch_bounds__(kBlock) void k_rg_start(int F, const double* __restrict__ r,
                                                     const double* __restrict__ D,
                                                     double* __restrict__ p, double* rr_parts,
                                                     Scalars* sc, StageArgs stage) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  if (stage.sc) {
    double rz_unused;
    if (stage_update<kBlock>(stage, red, rz_unused)) return;
  }
  double acc = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const double v = r[j];
    const double z = D ? v / D[j] : v;
    p[j] = z;
    acc += v * z;
  }
  store_block_partial<kBlock>(acc, rr_parts, blockIdx.x);
}

void launch_rg_start(int F, const double* r, const double* D, double* p, double* rr_parts,
                     Scalars* sc, const StageArgs* stage, hipStream_t s) {
  StageArgs st{};
  if (stage) st = *stage;
  k_rg_start<<<vec_grid(F), kBlock, 0, s>>>(F, r, D, p, rr_parts, sc, st);
}

__global__ __launch_bounds__(kBlock) void k_rg_step(int F, int first, const double* __restrict__ r,
                                                    const double* __restrict__ D,
                                                    double* __restrict__ e, double* __restrict__ res,
                                                    const double* __restrict__ p,
                                                    const double* __restrict__ q, const double* rr,
                                                    int n_rr, const double* pq, int n_pq,
                                                    double* rr_out, const Scalars* sc) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  const double rrv = sum_parts<kBlock>(rr, n_rr, red);
  const double pqv = sum_parts<kBlock>(pq, n_pq, red);
  // a vanishing residual (or a breakdown) leaves the rougher where it is
  const double alpha = (finite_pos(rrv) && finite_pos(pqv)) ? rrv / pqv : 0.0;
  double acc = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const double pj = p[j];
    e[j] = (first ? 0.0 : e[j]) + alpha * pj;
    const double v = (first ? r[j] : res[j]) - alpha * q[j];
    res[j] = v;
    acc += v * (D ? v / D[j] : v);
  }
  store_block_partial<kBlock>(acc, rr_out, blockIdx.x);
}

void launch_rg_step(int F, int first, const double* r, const double* D, double* e, double* res,
                    const double* p, const double* q, const double* rr, int n_rr, const double* pq,
                    int n_pq, double* rr_out, const Scalars* sc, hipStream_t s) {
  k_rg_step<<<vec_grid(F), kBlock, 0, s>>>(F, first, r, D, e, res, p, q, rr, n_rr, pq, n_pq, rr_out,
                                           sc);
}

__global__ __launch_bounds__(kBlock) void k_rg_dir(int F, const double* __restrict__ res,
                                                   const double* __restrict__ D,
                                                   double* __restrict__ p, const double* rr_new,
                                                   int n_new, const double* rr_old, int n_old,
                                                   const Scalars* sc) {
  if (sc->done) return;
  __shared__ double red[kBlock / 64];
  const double a = sum_parts<kBlock>(rr_new, n_new, red);
  const double b = sum_parts<kBlock>(rr_old, n_old, red);
  const double beta = finite_pos(b) ? a / b : 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock)
    p[j] = (D ? res[j] / D[j] : res[j]) + beta * p[j];
}

void launch_rg_dir(int F, const double* res, const double* D, double* p, const double* rr_new,
                   int n_new, const double* rr_old, int n_old, const Scalars* sc, hipStream_t s) {
  k_rg_dir<<<vec_grid(F), kBlock, 0, s>>>(F, res, D, p, rr_new, n_new, rr_old, n_old, sc);
}

// Noise-injection right-hand side: v = y + a xi1 (N) and b += c xi2 (F).
__global__ void k_noise_in(int N, const double* __restrict__ y, const double* __restrict__ xi1, double a,
                           double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) v[i] = y[i] + a * xi1[i];
}
void launch_noise_rhs_in(int N, const double* y, const double* xi1, double a, double* v, hipStream_t s) {
  if (N > 0) k_noise_in<<<cdiv(N, kBlock), kBlock, 0, s>>>(N, y, xi1, a, v);
}

__global__ void k_axpy_out(int F, double* __restrict__ b, const double* __restrict__ xi2, double c) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) b[j] += c * xi2[j];
}
void launch_axpy_out(int F, double* b, const double* xi2, double c, hipStream_t s) {
  if (F > 0) k_axpy_out<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, b, xi2, c);
}

// out = D in (row weights), in place allowed.
__global__ void k_row_scale(int N, const double* __restrict__ rw, const double* in, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = rw[i] * in[i];
}
void launch_row_scale(int N, const double* rw, const double* in, double* out, hipStream_t s) {
  if (N > 0) k_row_scale<<<cdiv(N, kBlock), kBlock, 0, s>>>(N, rw, in, out);
}

}  // namespace rr
