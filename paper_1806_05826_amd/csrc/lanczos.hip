// Prototype vectors of least-squares interpolation: the leading eigenvectors
// of X^T X (the principal directions of the feature space), which the paper
// computes with Arnoldi iterations.  X^T X is symmetric, so Arnoldi reduces to
// Lanczos; every new basis vector is orthogonalised against the whole basis
// twice (full reorthogonalisation keeps the basis orthonormal in FP64, which
// plain three-term Lanczos loses once Ritz values converge).  The Ritz pairs
// of the tridiagonal projection T_m come from a cyclic Jacobi
// eigendecomposition on the host (m <= 512); the Ritz vectors Q_m s_k are
// formed on the device.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "rr_device.h"

namespace rr {

// part[b * m + k] = block b's share of <Q_k, w>, k < m (rows of Q: F each)
__global__ __launch_bounds__(kBlock) void k_basis_dots(int F, int m, const double* __restrict__ Q,
                                                       const double* __restrict__ w, double* part) {
  __shared__ double red[kBlock / 64];
  for (int k = 0; k < m; ++k) {
    double s = 0.0;
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock)
      s += Q[(size_t)k * F + j] * w[j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * m + k] = s;
  }
}

// c[k] = sum over blocks of part[b * m + k], in block order
__global__ void k_basis_fold(int m, int nb, const double* __restrict__ part, double* c) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * m + k];
  c[k] = s;
}

// w -= sum_k c[k] Q_k
__global__ __launch_bounds__(kBlock) void k_basis_sub(int F, int m, const double* __restrict__ Q,
                                                      const double* __restrict__ c, double* w) {
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    double s = w[j];
    for (int k = 0; k < m; ++k) s -= c[k] * Q[(size_t)k * F + j];
    w[j] = s;
  }
}

// out = v * a
__global__ void k_scale_to(int F, const double* __restrict__ v, double a, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) out[j] = v[j] * a;
}

// out[j] = sum_k S[k] Q[k*F + j]   (a Ritz vector)
__global__ __launch_bounds__(kBlock) void k_combine(int F, int m, const double* __restrict__ Q,
                                                    const double* __restrict__ S, double* out) {
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += S[k] * Q[(size_t)k * F + j];
    out[j] = s;
  }
}

namespace {

// Symmetric eigendecomposition of a small dense matrix by cyclic Jacobi
// rotations (row-major n x n A, overwritten); ev[i] and column i of Z.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& ev, std::vector<double>& Z) {
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        // the rotation that zeroes a(p, q): t = tan(theta) from
        // cot(2 theta) = (a_qq - a_pp) / (2 a_pq), the smaller root
        const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double zkp = Z[(size_t)k * n + p], zkq = Z[(size_t)k * n + q];
          Z[(size_t)k * n + p] = c * zkp - s * zkq;
          Z[(size_t)k * n + q] = s * zkp + c * zkq;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = a(i, i);
}

}  // namespace

// The n_proto leading Ritz pairs of X^T X after `steps` Lanczos steps from a
// fixed start vector (SplitMix64(seed) entries in [0.5, 1.5) in the caller's
// feature order, normalised).  V: device [n_proto * F] in the caller's
// feature order; ev: host [n_proto], descending.
rr_status lanczos_prototypes(rr_handle* h, int n_proto, int steps, uint64_t seed, double* V, double* ev,
                             hipStream_t s) {
  const Sparse& X = h->X;
  const int F = X.F;
  const int m = std::min(steps, F);
  if (n_proto > m) return fail(RR_ERR_INVALID_ARG, "n_proto exceeds the Lanczos steps (or the features)");
  double *Q = nullptr, *w = nullptr, *u = nullptr, *part = nullptr, *c = nullptr, *S = nullptr,
         *tmp = nullptr;
  const int nb = std::min(vec_grid(F), 256);
  rr_status res = RR_OK;
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess && res == RR_OK) res = fail(RR_ERR_DEVICE, std::string("lanczos: ") + hipGetErrorString(e));
    return res == RR_OK;
  };
  if (ok(dmalloc(&Q, sizeof(double) * (size_t)(m + 1) * F)) && ok(dmalloc(&w, sizeof(double) * F)) &&
      ok(dmalloc(&u, sizeof(double) * std::max(1, X.N))) && ok(dmalloc(&part, sizeof(double) * (size_t)nb * (m + 1))) &&
      ok(dmalloc(&c, sizeof(double) * (m + 1))) && ok(dmalloc(&S, sizeof(double) * (m + 1))) &&
      ok(dmalloc(&tmp, sizeof(double) * F))) {
    // q0 in internal order
    std::vector<double> v0(F);
    uint64_t st = seed;
    double ss = 0.0;
    for (int j = 0; j < F; ++j) {
      v0[j] = (double)(splitmix64_next(st) >> 11) * (1.0 / 9007199254740992.0) + 0.5;
      ss += v0[j] * v0[j];
    }
    for (auto& x : v0) x /= std::sqrt(ss);
    ok(hipMemcpyAsync(tmp, v0.data(), sizeof(double) * F, hipMemcpyHostToDevice, s));
    launch_gather(Q, tmp, h->fperm, F, s);
    std::vector<double> alpha, beta, cv(m + 1);
    int mm = 0;   // basis size reached
    auto dots = [&](int rows, const double* vec) {   // c[0, rows) = Q[0, rows)^T vec
      k_basis_dots<<<nb, kBlock, 0, s>>>(F, rows, Q, vec, part);
      k_basis_fold<<<cdiv(rows, 64), 64, 0, s>>>(rows, nb, part, c);
    };
    for (int j = 0; j < m && res == RR_OK; ++j) {
      const double* qj = Q + (size_t)j * F;
      // w = X^T (X q_j)
      launch_csr(X, qj, u, nullptr, s);
      Epi e{};
      e.out = w;
      launch_csc(X, u, EPI_STORE, e, nullptr, s);
      // full reorthogonalisation, twice; alpha_j = <q_j, w> from the first
      double a = 0.0;
      for (int pass = 0; pass < 2 && res == RR_OK; ++pass) {
        dots(j + 1, w);
        if (pass == 0) {
          ok(hipMemcpyAsync(cv.data(), c, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s));
          ok(hipStreamSynchronize(s));
          a = cv[j];
        }
        k_basis_sub<<<nb, kBlock, 0, s>>>(F, j + 1, Q, c, w);
      }
      // beta_j = ||w||
      k_basis_dots<<<nb, kBlock, 0, s>>>(F, 1, w, w, part);
      k_basis_fold<<<1, 64, 0, s>>>(1, nb, part, c);
      double bb = 0.0;
      ok(hipMemcpyAsync(&bb, c, sizeof(double), hipMemcpyDeviceToHost, s));
      ok(hipStreamSynchronize(s));
      alpha.push_back(a);
      mm = j + 1;
      const double b = std::sqrt(std::max(bb, 0.0));
      if (!(b > 1e-12 * std::max(1.0, std::fabs(a))) || j + 1 == m) break;   // invariant subspace or done
      beta.push_back(b);
      k_scale_to<<<cdiv(F, 256), 256, 0, s>>>(F, w, 1.0 / b, Q + (size_t)(j + 1) * F);
    }
    if (res == RR_OK && mm < n_proto)
      res = fail(RR_ERR_INVALID_ARG, "the Krylov space closed before n_proto directions (rank of X)");
    if (res == RR_OK) {
      // T_mm: alpha on the diagonal, beta beside it (the reorthogonalised
      // projection Q^T A Q, tridiagonal up to rounding)
      std::vector<double> T((size_t)mm * mm, 0.0), evs, Z;
      for (int i = 0; i < mm; ++i) T[(size_t)i * mm + i] = alpha[i];
      for (int i = 0; i + 1 < mm; ++i) T[(size_t)i * mm + i + 1] = T[(size_t)(i + 1) * mm + i] = beta[i];
      jacobi_eigen(mm, T, evs, Z);
      std::vector<int> ord(mm);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return evs[x] > evs[y]; });
      std::vector<double> sk(mm);
      for (int k = 0; k < n_proto && res == RR_OK; ++k) {
        const int col = ord[k];
        for (int i = 0; i < mm; ++i) sk[i] = Z[(size_t)i * mm + col];
        // a fixed sign: the largest component of the Ritz vector's
        // coefficients positive
        int big = 0;
        for (int i = 1; i < mm; ++i)
          if (std::fabs(sk[i]) > std::fabs(sk[big])) big = i;
        if (sk[big] < 0)
          for (auto& x : sk) x = -x;
        ev[k] = evs[col];
        ok(hipMemcpyAsync(S, sk.data(), sizeof(double) * mm, hipMemcpyHostToDevice, s));
        k_combine<<<nb, kBlock, 0, s>>>(F, mm, Q, S, tmp);
        launch_gather(V + (size_t)k * F, tmp, h->finv, F, s);   // internal -> caller order
        ok(hipStreamSynchronize(s));
      }
    }
  }
  (void)hipStreamSynchronize(s);
  dev_free(Q);
  dev_free(w);
  dev_free(u);
  dev_free(part);
  dev_free(c);
  dev_free(S);
  dev_free(tmp);
  if (res == RR_OK) RR_HIP(hipGetLastError());
  return res;
}

}  // namespace rr
