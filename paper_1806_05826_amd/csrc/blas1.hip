// Fused vector kernels of the PCG iteration (the x/r updates and the
// scalars of the flexible-CG algorithm's update steps, specialised to a
// fixed preconditioner).  Every reduction finishes in the last block to
// arrive, in block order, so scalars stay on the device and results are
// bitwise reproducible run to run.
#include "rr_device.h"

namespace rr {

// x = 0, r = b, p = 0, ||b||^2, ||x_ref||^2 and the first smoother step.
__global__ __launch_bounds__(kBlock) void k_pcg_init(int F, const double* __restrict__ b,
                                                     double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     double* __restrict__ p,
                                                     double* __restrict__ z,
                                                     double* __restrict__ e1,
                                                     const double* __restrict__ D,
                                                     const double* __restrict__ xref,
                                                     double omega, int kind, Scalars* sc,
                                                     double* partials, double* history) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (j < F) {
    const double bj = b[j];
    x[j] = 0.0;
    r[j] = bj;
    p[j] = 0.0;
    v[0] = bj * bj;
    if (xref) v[1] = xref[j] * xref[j];
    if (kind == PK_JACOBI) {
      const double zj = bj / D[j];
      z[j] = zj;
      v[2] = bj * zj;
    } else if (kind == PK_NONE) {
      z[j] = bj;
      v[2] = bj * bj;
    } else if (kind == PK_VCYCLE) {
      e1[j] = (omega * bj) / D[j];
    }
  }
  double tot[3];
  if (grid_finish<3>(v, partials, 0, gridDim.x, &sc->ticket, tot) && threadIdx.x == 0) {
    sc->bb = tot[0];
    sc->ref2 = tot[1];
    sc->tol2 *= tot[0];
    sc->errtol2 *= tot[1];
    sc->iter = 0;
    if (history) history[0] = (tot[0] > 0.0) ? 1.0 : 0.0;
    if (!(tot[0] > 0.0)) {
      sc->done = 1;
      sc->status = (tot[0] == 0.0) ? RR_OK : RR_ERR_BREAKDOWN;
      sc->true_rr = 0.0;
    } else if (kind == PK_JACOBI || kind == PK_NONE) {
      finish_beta(sc, tot[2]);
    }
  }
}

void launch_pcg_init(int F, const double* b, double* x, double* r, double* p, double* z,
                     double* e1, const double* D, const double* xref, double omega, int kind,
                     Scalars* sc, double* partials, double* history, hipStream_t s) {
  k_pcg_init<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, b, x, r, p, z, e1, D, xref, omega, kind, sc,
                                                partials, history);
}

// x += alpha p; r -= alpha q; ||r||^2; optional error; next smoother input.
__global__ __launch_bounds__(kBlock) void k_pcg_update(
    int F, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ z, double* __restrict__ e1,
    const double* __restrict__ D, const double* __restrict__ xref, double omega, int kind,
    Scalars* sc, double* partials, double* history) {
  if (sc->done) return;
  const double alpha = sc->alpha;
  const int j = blockIdx.x * kBlock + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (j < F) {
    const double xj = x[j] + alpha * p[j];
    const double rj = r[j] - alpha * q[j];
    x[j] = xj;
    r[j] = rj;
    v[0] = rj * rj;
    if (xref) {
      const double d = xj - xref[j];
      v[1] = d * d;
    }
    if (kind == PK_JACOBI) {
      const double zj = rj / D[j];
      z[j] = zj;
      v[2] = rj * zj;
    } else if (kind == PK_NONE) {
      z[j] = rj;
      v[2] = rj * rj;
    } else if (kind == PK_VCYCLE) {
      e1[j] = (omega * rj) / D[j];
    }
  }
  double tot[3];
  if (grid_finish<3>(v, partials, 0, gridDim.x, &sc->ticket, tot) && threadIdx.x == 0) {
    const double rr = tot[0];
    sc->rr = rr;
    sc->ee = tot[1];
    const int it = ++sc->iter;
    if (history) history[it] = sqrt(rr / sc->bb);
    if (!(rr == rr)) {
      sc->status = RR_ERR_BREAKDOWN;
      sc->done = 1;
      return;
    }
    if (sc->fixed > 0) {
      if (it >= sc->fixed) {
        sc->status = RR_OK;
        sc->done = 1;
      }
    } else if (rr <= sc->tol2 || (sc->use_err && tot[1] <= sc->errtol2)) {
      sc->status = RR_OK;
      sc->done = 1;
    } else if (it >= sc->limit) {
      sc->done = 1;
    }
    if (!sc->done && (kind == PK_JACOBI || kind == PK_NONE)) finish_beta(sc, tot[2]);
  }
}

void launch_pcg_update(int F, double* x, double* r, const double* p, const double* q,
                       double* z, double* e1, const double* D, const double* xref,
                       double omega, int kind, Scalars* sc, double* partials, double* history,
                       hipStream_t s) {
  k_pcg_update<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, x, r, p, q, z, e1, D, xref, omega, kind,
                                                  sc, partials, history);
}

__global__ __launch_bounds__(kBlock) void k_pupdate(int F, double* __restrict__ p,
                                                    const double* __restrict__ z,
                                                    const Scalars* sc) {
  if (sc->done) return;
  const double beta = sc->beta;
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < F) p[j] = z[j] + beta * p[j];
}

void launch_pupdate(int F, double* p, const double* z, Scalars* sc, hipStream_t s) {
  k_pupdate<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, p, z, sc);
}

// Prolongation: out = e1 + P yc (V-cycle), or the additive form
// z = w D^-1 r + P yc with <r,z> -> beta.
__global__ __launch_bounds__(kBlock) void k_prolong(int F, const int* __restrict__ labels,
                                                    const double* __restrict__ cscale,
                                                    const double* __restrict__ yc,
                                                    const double* __restrict__ e1,
                                                    double* __restrict__ out,
                                                    const double* __restrict__ r,
                                                    const double* __restrict__ D, double omega,
                                                    int additive, Scalars* sc,
                                                    double* partials) {
  if (sc && sc->done) return;
  const int j = blockIdx.x * kBlock + threadIdx.x;
  double v[1] = {0.0};
  if (j < F) {
    const int s = labels[j];
    const double corr = cscale[s] * yc[s];
    if (additive) {
      const double rj = r[j];
      const double zj = (omega * rj) / D[j] + corr;
      out[j] = zj;
      v[0] = rj * zj;
    } else {
      out[j] = e1[j] + corr;
    }
  }
  if (additive && sc) {
    double tot[1];
    if (grid_finish<1>(v, partials, 0, gridDim.x, &sc->ticket, tot) && threadIdx.x == 0)
      finish_beta(sc, tot[0]);
  }
}

void launch_prolong(int F, const int* labels, const double* cscale, const double* yc,
                    const double* e1, double* out, const double* r, const double* D,
                    double omega, int additive, Scalars* sc, double* partials, hipStream_t s) {
  k_prolong<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, labels, cscale, yc, e1, out, r, D, omega,
                                               additive, sc, partials);
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

__global__ void k_axpby(long long n, double a, const double* x, double b, double* y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
void launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n > 0) k_axpby<<<cdiv(n, kBlock), kBlock, 0, s>>>(n, a, x, b, y);
}

__global__ __launch_bounds__(kBlock) void k_dot(long long n, const double* x, const double* y,
                                                double* out, double* partials,
                                                unsigned* ticket) {
  double v[1] = {0.0};
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    v[0] += x[i] * y[i];
  double tot[1];
  if (grid_finish<1>(v, partials, 0, gridDim.x, ticket, tot) && threadIdx.x == 0) *out = tot[0];
}
void launch_dot(long long n, const double* x, const double* y, double* out, double* partials,
                unsigned* ticket, hipStream_t s) {
  const int grid = std::max(1, std::min(1024, cdiv(n, kBlock)));
  k_dot<<<grid, kBlock, 0, s>>>(n, x, y, out, partials, ticket);
}

// y = A x, A row-major n x n: one wave per row.
__global__ __launch_bounds__(kBlock) void k_gemv(int n, const double* __restrict__ A,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y, const int* done) {
  if (is_done(done)) return;
  const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* a = A + (size_t)row * n;
  double acc = 0.0;
  for (int c = lane; c < n; c += 64) acc += a[c] * x[c];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[row] = acc;
}
void launch_gemv(int n, const double* A, const double* x, double* y, const int* done,
                 hipStream_t s) {
  if (n > 0) k_gemv<<<cdiv(n, kBlock / 64), kBlock, 0, s>>>(n, A, x, y, done);
}

}  // namespace rr
