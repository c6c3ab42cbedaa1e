// Coarse level per lambda: A_c = K + lambda I (the Galerkin coarse matrix
// P^T A P = X_c^T X_c + lambda I, since P^T P = I; with least-squares
// interpolation P^T P is the diagonal G and A_c = K + lambda G), its Cholesky factor L
// (the coarse solver of the paper's experiments) and A_c^-1 = L^-T L^-1,
// kept explicitly so that each coarse solve is one matrix-vector product on
// the whole GPU instead of two sequential triangular solves.  All FP64.
#include <vector>

#include "rr_device.h"

namespace rr {

constexpr int NB = 32;   // Cholesky panel width

__global__ void k_form_ac(int n, const double* __restrict__ K, double lam, const double* __restrict__ g,
                          double* __restrict__ A) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n) return;
  const int r = (int)(i / n), c = (int)(i % n);
  A[i] = K[i] + (r == c ? (g ? lam * g[r] : lam) : 0.0);
}

// Unblocked Cholesky of the nb x nb diagonal block at (k0, k0), in LDS.
__global__ __launch_bounds__(kBlock) void k_potrf_diag(double* A, int n, int k0, int nb, int* flag) {
  __shared__ double a[NB][NB + 1];
  for (int t = threadIdx.x; t < nb * nb; t += kBlock) {
    const int i = t / nb, j = t % nb;
    a[i][j] = (j <= i) ? A[(size_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (threadIdx.x == 0) {
      double d = a[j][j];
      if (!(d > 0.0) || !(d < __builtin_inf())) {
        atomicOr(flag, 1);
        d = 1.0;
      }
      a[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < nb; i += kBlock) a[i][j] /= a[j][j];
    __syncthreads();
    const int m = nb - j - 1;   // trailing size
    for (int t = threadIdx.x; t < m * m; t += kBlock) {
      const int i = j + 1 + t / m, l = j + 1 + t % m;
      if (l <= i) a[i][l] -= a[i][j] * a[l][j];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nb * nb; t += kBlock) {
    const int i = t / nb, j = t % nb;
    if (j <= i) A[(size_t)(k0 + i) * n + k0 + j] = a[i][j];
  }
}

// Rows below the diagonal block: L_i = A_i L_kk^-T (one thread per row).
__global__ __launch_bounds__(kBlock) void k_trsm_panel(double* A, int n, int k0, int nb) {
  __shared__ double l[NB][NB + 1];
  for (int t = threadIdx.x; t < nb * nb; t += kBlock) {
    const int i = t / nb, j = t % nb;
    l[i][j] = (j <= i) ? A[(size_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  const int row = k0 + nb + blockIdx.x * kBlock + threadIdx.x;
  if (row >= n) return;
  double x[NB];
  double* a = A + (size_t)row * n + k0;
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = (j < nb) ? a[j] : 0.0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nb) {
      double s = x[j];
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < j) s -= x[q] * l[j][q];
      x[j] = s / l[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < nb) a[j] = x[j];
}

// Trailing update A_ij -= sum_q L_iq L_jq over the panel, lower tiles only.
__global__ __launch_bounds__(kBlock) void k_syrk(double* A, int n, int k0, int nb) {
  __shared__ double li[NB][NB + 1];
  __shared__ double lj[NB][NB + 1];
  // blockIdx.x enumerates lower-triangular tile pairs (ti >= tj)
  const int b = blockIdx.x;
  int ti = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int tj = b - ti * (ti + 1) / 2;
  const int base = k0 + nb;
  const int r0 = base + ti * NB, c0 = base + tj * NB;
  for (int t = threadIdx.x; t < NB * NB; t += kBlock) {
    const int i = t / NB, q = t % NB;
    li[i][q] = (r0 + i < n && q < nb) ? A[(size_t)(r0 + i) * n + k0 + q] : 0.0;
    lj[i][q] = (c0 + i < n && q < nb) ? A[(size_t)(c0 + i) * n + k0 + q] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < NB * NB; t += kBlock) {
    const int i = t / NB, j = t % NB;
    const int gi = r0 + i, gj = c0 + j;
    if (gi < n && gj < n && gj <= gi) {
      double s = 0.0;
#pragma unroll 8
      for (int q = 0; q < NB; ++q) s += li[i][q] * lj[j][q];
      A[(size_t)gi * n + gj] -= s;
    }
  }
}

__global__ void k_lower_and_transpose(int n, const double* A, double* L, double* Lt) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  const double v = (j <= i) ? A[t] : 0.0;
  L[t] = v;
  Lt[(size_t)j * n + i] = v;
}

// Row s of W = (L^-1)^T, i.e. column s of L^-1: forward substitution with the
// transposed factor so that every step reads a contiguous row.
__global__ __launch_bounds__(kBlock) void k_trinv_cols(int n, const double* __restrict__ Lt,
                                                       double* __restrict__ W) {
  extern __shared__ double w[];
  const int s = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += kBlock) w[i] = (i == s) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = s; j < n; ++j) {
    const double* lj = Lt + (size_t)j * n;
    const double wj = w[j] / lj[j];
    __syncthreads();
    if (threadIdx.x == 0) w[j] = wj;
    for (int i = j + 1 + threadIdx.x; i < n; i += kBlock) w[i] -= lj[i] * wj;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += kBlock) W[(size_t)s * n + i] = w[i];
}

// C = W W^T (n x n), 64 x 64 tiles, 4 x 4 outputs per thread.
__global__ __launch_bounds__(kBlock) void k_gemm_nt(int n, const double* __restrict__ W,
                                                    double* __restrict__ C) {
  constexpr int T = 64, KT = 16;
  __shared__ double a[KT][T + 1];
  __shared__ double bsh[KT][T + 1];
  const int r0 = blockIdx.y * T, c0 = blockIdx.x * T;
  const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < n; k0 += KT) {
    for (int t = threadIdx.x; t < T * KT; t += kBlock) {
      const int i = t / KT, q = t % KT;
      a[q][i] = (r0 + i < n && k0 + q < n) ? W[(size_t)(r0 + i) * n + k0 + q] : 0.0;
      bsh[q][i] = (c0 + i < n && k0 + q < n) ? W[(size_t)(c0 + i) * n + k0 + q] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KT; ++q) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = a[q][tr + u];
        bv[u] = bsh[q][tc + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = r0 + tr + u, gj = c0 + tc + v;
      if (gi < n && gj < n) C[(size_t)gi * n + gj] = acc[u][v];
    }
}

// ---- K = Q diag(ev) Q^T by parallel cyclic Jacobi ---------------------------
// The coarse solve of the Bayesian-regression experiments uses the SVD of
// X_c = X P, whose right singular vectors and squared singular values are
// the eigenvectors and eigenvalues of K = X_c^T X_c; with them,
// A_c(lam)^-1 = Q diag(1 / (ev + lam)) Q^T for every lam without a new
// factorization.  A sweep visits every pair (p, q) once, in m - 1 rounds of
// m / 2 disjoint pairs (m = n rounded up to even; the circle ordering, with
// the index m - 1 a dummy when n is odd).  Rotation (p, q) zeroes a_pq
// (the symmetric 2 x 2 Schur step): with tau = (a_qq - a_pp) / (2 a_pq),
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1 / sqrt(1 + t^2), s = t c,
// A <- J^T A J and Q <- Q J, J the identity but for J_pp = J_qq = c,
// J_pq = s, J_qp = -s.  A round computes every pair's rotation from its own
// two rows, then updates rows, then columns (the pairs are disjoint, so
// these updates do not interfere).
__device__ inline void circle_pair(int m, int round, int k, int* p, int* q) {
  auto at = [&](int i) { return i == 0 ? m - 1 : (round + i - 1) % (m - 1); };
  const int a = at(k), b = at(m - 1 - k);
  *p = min(a, b);
  *q = max(a, b);
}

__global__ __launch_bounds__(kBlock) void k_jacobi_rows(int n, int m, int round, double* __restrict__ A,
                                                        double2* __restrict__ cs) {
  const int k = blockIdx.x;
  int p, q;
  circle_pair(m, round, k, &p, &q);
  if (q >= n) {   // the dummy index of an odd n
    if (threadIdx.x == 0) cs[k] = make_double2(1.0, 0.0);
    return;
  }
  double* ap = A + (size_t)p * n;
  double* aq = A + (size_t)q * n;
  const double apq = ap[q], app = ap[p], aqq = aq[q];
  double c = 1.0, sn = 0.0;
  if (apq != 0.0) {
    const double tau = (aqq - app) / (2.0 * apq);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + t * t);
    sn = t * c;
  }
  __syncthreads();   // every thread has read the pivot entries before any write
  if (threadIdx.x == 0) cs[k] = make_double2(c, sn);
  if (sn == 0.0) return;
  for (int j = threadIdx.x; j < n; j += kBlock) {
    const double x = ap[j], y = aq[j];
    ap[j] = c * x - sn * y;
    aq[j] = sn * x + c * y;
  }
}

// Column rotations of one round, one block per row i of A and of Q: every
// column j has exactly one partner in the round, so the block stages the row
// in LDS and writes each entry from itself and its partner (coalesced).
__device__ inline int circle_pos(int m, int round, int j) { return j == m - 1 ? 0 : (j - round + (m - 1)) % (m - 1) + 1; }

__global__ __launch_bounds__(kBlock) void k_jacobi_cols(int n, int m, int round, double* __restrict__ A,
                                                        double* __restrict__ Q, const double2* __restrict__ cs) {
  extern __shared__ double row[];   // [2 n]: row i of A, then of Q
  const int i = blockIdx.x;
  double* ai = A + (size_t)i * n;
  double* qi = Q + (size_t)i * n;
  for (int j = threadIdx.x; j < n; j += kBlock) {
    row[j] = ai[j];
    row[n + j] = qi[j];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += kBlock) {
    const int pos = circle_pos(m, round, j);
    const int ppos = m - 1 - pos;
    const int partner = ppos == 0 ? m - 1 : (round + ppos - 1) % (m - 1);
    if (partner >= n) continue;   // paired with the dummy index: untouched
    const double2 r = cs[min(pos, ppos)];
    if (r.y == 0.0) continue;
    const bool is_p = j < partner;   // (p, q) = (min, max)
    const double xa = row[j], ya = row[partner];
    const double xq = row[n + j], yq = row[n + partner];
    // new column p = c col_p - s col_q, new column q = s col_p + c col_q
    if (is_p) {
      ai[j] = (i == partner) ? 0.0 : r.x * xa - r.y * ya;
      qi[j] = r.x * xq - r.y * yq;
    } else {
      ai[j] = (i == partner) ? 0.0 : r.y * ya + r.x * xa;
      qi[j] = r.y * yq + r.x * xq;
    }
  }
}

// sum of the squared off-diagonal entries (one partial per block) and of
// all entries
__global__ __launch_bounds__(kBlock) void k_offdiag(int n, const double* __restrict__ A, double* parts) {
  double off = 0.0, all = 0.0;
  const long long nn = (long long)n * n;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nn; i += (long long)gridDim.x * kBlock) {
    const double a = A[i];
    all += a * a;
    if (i / n != i % n) off += a * a;
  }
  __shared__ double red[kBlock / 64];
  const double o = block_sum(off, red);
  const double t = block_sum(all, red);
  if (threadIdx.x == 0) {
    parts[2 * blockIdx.x] = o;
    parts[2 * blockIdx.x + 1] = t;
  }
}

__global__ void k_identity(int n, double* Q) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (long long)n * n) Q[i] = (i / n == i % n) ? 1.0 : 0.0;
}

__global__ void k_diag(int n, const double* A, double* ev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ev[i] = A[(size_t)i * n + i];
}

// Setup only: h->eig_q, h->eig_v from h->K.  *sweeps receives the sweeps run.
rr_status coarse_eigen(rr_handle* h, int* sweeps, hipStream_t s) {
  const int n = h->FC;
  if (n <= 0) return fail(RR_ERR_INVALID_ARG, "no coarse level (n_clusters = 0)");
  const long long nn = (long long)n * n;
  const int m = n + (n & 1);
  if (!h->eig_q) RR_HIP(dmalloc(&h->eig_q, sizeof(double) * nn));
  if (!h->eig_v) RR_HIP(dmalloc(&h->eig_v, sizeof(double) * n));
  double* A = h->chol_work;   // FC^2 scratch for the rotated K
  double2* cs = nullptr;
  double* parts = nullptr;
  constexpr int kOffBlocks = 256;
  RR_HIP(dmalloc(&cs, sizeof(double2) * (m / 2)));
  RR_HIP(dmalloc(&parts, sizeof(double) * 2 * kOffBlocks));
  RR_HIP(hipMemcpyAsync(A, h->K, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
  k_identity<<<cdiv(nn, kBlock), kBlock, 0, s>>>(n, h->eig_q);
  std::vector<double> hp(2 * kOffBlocks);
  rr_status st = RR_OK;
  int sw = 0;
  double off_prev = -1.0;
  for (; sw < kMaxJacobiSweeps; ++sw) {
    k_offdiag<<<kOffBlocks, kBlock, 0, s>>>(n, A, parts);
    if (hipMemcpyAsync(hp.data(), parts, sizeof(double) * 2 * kOffBlocks, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = fail(RR_ERR_DEVICE, "eigen: reading the off-diagonal norm");
      break;
    }
    double off = 0.0, all = 0.0;
    for (int b = 0; b < kOffBlocks; ++b) {
      off += hp[2 * b];
      all += hp[2 * b + 1];
    }
    // off-diagonal Frobenius norm <= 1e-15 of the whole, or no longer
    // shrinking once below 1e-11 of it (the rounding floor)
    if (off <= 1e-30 * all) break;
    if (off_prev >= 0.0 && off <= 1e-22 * all && off > 0.25 * off_prev) break;
    off_prev = off;
    for (int r = 0; r < m - 1; ++r) {
      k_jacobi_rows<<<m / 2, kBlock, 0, s>>>(n, m, r, A, cs);
      k_jacobi_cols<<<n, kBlock, sizeof(double) * 2 * n, s>>>(n, m, r, A, h->eig_q, cs);
    }
  }
  if (st == RR_OK && sw == kMaxJacobiSweeps) st = fail(RR_ERR_NOT_CONVERGED, "eigen: Jacobi sweeps did not converge");
  if (st == RR_OK) k_diag<<<cdiv(n, kBlock), kBlock, 0, s>>>(n, A, h->eig_v);
  (void)hipStreamSynchronize(s);
  (void)dev_free(cs);
  (void)dev_free(parts);
  RR_TRY(st);
  RR_HIP(hipGetLastError());
  *sweeps = sw;
  return RR_OK;
}

// W = Q diag(1 / sqrt(ev + lam)); a non-positive ev + lam sets *bad.
__global__ void k_eig_scale(int n, const double* __restrict__ Q, const double* __restrict__ ev, double lam,
                            double* __restrict__ W, int* bad) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n) return;
  const double d = ev[i % n] + lam;
  if (!(d > 0.0)) {
    *bad = 1;
    W[i] = 0.0;
    return;
  }
  W[i] = Q[i] / sqrt(d);
}

// A_c(lam)^-1 = W W^T from the eigendecomposition (no Cholesky factor).
rr_status coarse_from_eigen(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s) {
  const int n = h->FC;
  const long long nn = (long long)n * n;
  double* W = h->chol_work;
  RR_HIP(hipMemsetAsync(h->chol_flag, 0, sizeof(int), s));
  k_eig_scale<<<cdiv(nn, kBlock), kBlock, 0, s>>>(n, h->eig_q, h->eig_v, lam, W, h->chol_flag);
  dim3 grid(cdiv(n, 64), cdiv(n, 64));
  k_gemm_nt<<<grid, kBlock, 0, s>>>(n, W, slot.Ainv);
  int flag = 0;
  RR_HIP(hipMemcpyAsync(&flag, h->chol_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  if (flag) return fail(RR_ERR_BREAKDOWN, "coarse eigenvalue + lambda is not positive");
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status coarse_factor(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s) {
  const int n = h->FC;
  if (n <= 0) return fail(RR_ERR_INVALID_ARG, "no coarse level (n_clusters = 0)");
  const long long nn = (long long)n * n;
  double* A = h->chol_work;
  RR_HIP(hipMemsetAsync(h->chol_flag, 0, sizeof(int), s));
  k_form_ac<<<cdiv(nn, kBlock), kBlock, 0, s>>>(n, h->K, lam, h->pgram, A);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = std::min(NB, n - k0);
    k_potrf_diag<<<1, kBlock, 0, s>>>(A, n, k0, nb, h->chol_flag);
    const int rest = n - k0 - nb;
    if (rest > 0) {
      k_trsm_panel<<<cdiv(rest, kBlock), kBlock, 0, s>>>(A, n, k0, nb);
      const int T = cdiv(rest, NB);
      k_syrk<<<T * (T + 1) / 2, kBlock, 0, s>>>(A, n, k0, nb);
    }
  }
  double* Lt = h->chol_work + nn;   // second half of the scratch
  k_lower_and_transpose<<<cdiv(nn, kBlock), kBlock, 0, s>>>(n, A, slot.L, Lt);
  int flag = 0;
  RR_HIP(hipMemcpyAsync(&flag, h->chol_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  if (flag) return fail(RR_ERR_BREAKDOWN, "coarse matrix is not numerically positive definite");
  double* W = A;   // reuse the factor scratch for L^-T
  k_trinv_cols<<<n, kBlock, sizeof(double) * n, s>>>(n, Lt, W);
  dim3 grid(cdiv(n, 64), cdiv(n, 64));
  k_gemm_nt<<<grid, kBlock, 0, s>>>(n, W, slot.Ainv);
  RR_HIP(hipGetLastError());
  return RR_OK;
}

}  // namespace rr
