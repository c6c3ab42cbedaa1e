// Coarse level per lambda: A_c = K + lambda I (the Galerkin coarse matrix
// P^T A P = X_c^T X_c + lambda I, since P^T P = I), its Cholesky factor L
// (the coarse solver of the paper's experiments) and A_c^-1 = L^-T L^-1,
// kept explicitly so that each coarse solve is one matrix-vector product on
// the whole GPU instead of two sequential triangular solves.  All FP64.
#include "rr_device.h"

namespace rr {

constexpr int NB = 32;   // Cholesky panel width

__global__ void k_form_ac(int n, const double* __restrict__ K, double lam, double* __restrict__ A) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n) return;
  const int r = (int)(i / n), c = (int)(i % n);
  A[i] = K[i] + (r == c ? lam : 0.0);
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

rr_status coarse_factor(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s) {
  const int n = h->FC;
  if (n <= 0) return fail(RR_ERR_INVALID_ARG, "no coarse level (n_clusters = 0)");
  const long long nn = (long long)n * n;
  double* A = h->chol_work;
  RR_HIP(hipMemsetAsync(h->chol_flag, 0, sizeof(int), s));
  k_form_ac<<<cdiv(nn, kBlock), kBlock, 0, s>>>(n, h->K, lam, A);
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
