// Least-squares interpolation (the least-squares interpolation subsection of
// the paper's method section).  Every fine feature j is interpolated from
// the coarse feature r of its cluster alone, so row j of P holds one weight
//     p_j = sum_k eta_k v_k(j) v_k(r) / sum_k eta_k v_k(r)^2,
// the minimiser of sum_k eta_k (v_k(j) - p_j v_k(r))^2 over the prototype
// vectors v_k, with eta_k = <(X^T X + beta I) v_k, v_k> from the operator's
// own passes.  The coarse feature of a cluster is the caller's choice or its
// member of lowest caller index (the leader, under leader-follower
// clustering); a cluster whose coarse feature has zero weighted energy keeps
// plain aggregation (p_j = 1; the coarse correction is blind to the scale of
// a column of P).  P^T P becomes diag(sum of p_j^2 per cluster), which the
// coarse matrix carries as lambda times that diagonal.
#include <climits>

#include "rr_device.h"

namespace rr {

namespace {

__global__ void k_fill_rep(int n, int* a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = INT_MAX;
}

// rep[s] = the lowest caller index among the members of cluster s
__global__ void k_rep_min(int F, const int* __restrict__ labels, const int* __restrict__ fperm,
                          int* rep) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) atomicMin(&rep[labels[j]], fperm[j]);
}

// caller's coarse features -> internal indices; bad = 1 for one out of range
// or outside its cluster
__global__ void k_rep_internal(int fc, int F, const int* __restrict__ rep_caller,
                               const int* __restrict__ finv, const int* __restrict__ labels,
                               int* __restrict__ rep_int, int* bad) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= fc) return;
  const int r = rep_caller[c];
  if (r < 0 || r >= F) {
    rep_int[c] = 0;
    *bad = 1;
    return;
  }
  const int i = finv[r];
  rep_int[c] = i;
  if (labels[i] != c) *bad = 1;
}

// eta = <t + beta v, v> in one workgroup, fixed order
__global__ __launch_bounds__(kBlock) void k_energy(int F, const double* __restrict__ t,
                                                   const double* __restrict__ v, double beta,
                                                   double* eta) {
  __shared__ double red[kBlock];
  double a = 0.0;
  for (int i = threadIdx.x; i < F; i += kBlock) a += (t[i] + beta * v[i]) * v[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *eta = red[0];
}

// den[s] = sum_k eta_k v_k(r_s)^2 (prototype k at Vi + k F, internal order)
__global__ void k_ls_den(int fc, int F, int K, const double* __restrict__ Vi,
                         const double* __restrict__ eta, const int* __restrict__ rep_int,
                         double* __restrict__ den) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= fc) return;
  const int r = rep_int[c];
  double d = 0.0;
  for (int k = 0; k < K; ++k) {
    const double x = Vi[(size_t)k * F + r];
    d += eta[k] * (x * x);
  }
  den[c] = d;
}

__global__ void k_ls_weights(int F, int K, const double* __restrict__ Vi,
                             const double* __restrict__ eta, const int* __restrict__ labels,
                             const int* __restrict__ rep_int, const double* __restrict__ den,
                             double* __restrict__ pw, int* bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F) return;
  const int l = labels[j];
  const double dn = den[l];
  if (dn == 0.0) {
    pw[j] = 1.0;
    return;
  }
  const int r = rep_int[l];
  double n = 0.0;
  for (int k = 0; k < K; ++k) n += eta[k] * (Vi[(size_t)k * F + j] * Vi[(size_t)k * F + r]);
  const double p = n / dn;
  pw[j] = p;
  if (!(p - p == 0.0)) *bad = 1;   // NaN or infinite
}

__global__ void k_perm_vals(int F, const int* __restrict__ perm, const double* __restrict__ pw,
                            double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < F) out[k] = pw[perm[k]];
}

}  // namespace

void free_interpolation(rr_handle* h) {
  (void)dev_free(h->lsw);
  (void)dev_free(h->lsw_perm);
  (void)dev_free(h->pgram);
  h->lsw = h->lsw_perm = h->pgram = nullptr;
}

rr_status set_interpolation(rr_handle* h, const double* V, int K, double beta, const int* rep,
                            double* p_out, hipStream_t s) {
  const int F = h->X.F, N = h->X.N, fc = h->FC;
  if (!V) {   // back to the adjusted square-root average
    if (h->lsw) {
      free_interpolation(h);
      RR_TRY(build_coarse_gram(h, s));
    }
    return RR_OK;
  }
  double *Vi = nullptr, *eta = nullptr, *t = nullptr, *u = nullptr, *den = nullptr;
  double *pw = nullptr, *pw_perm = nullptr, *pgram = nullptr;
  int *rep_c = nullptr, *rep_int = nullptr, *bad = nullptr;
  auto release = [&]() {
    (void)dev_free(Vi); (void)dev_free(eta); (void)dev_free(t); (void)dev_free(u);
    (void)dev_free(den); (void)dev_free(rep_c); (void)dev_free(rep_int); (void)dev_free(bad);
  };
  auto drop_new = [&]() {
    (void)dev_free(pw); (void)dev_free(pw_perm); (void)dev_free(pgram);
  };
  bool ok = dmalloc(&Vi, sizeof(double) * (size_t)K * F) == hipSuccess &&
            dmalloc(&eta, sizeof(double) * K) == hipSuccess &&
            dmalloc(&t, sizeof(double) * F) == hipSuccess &&
            dmalloc(&u, sizeof(double) * std::max(1, N)) == hipSuccess &&
            dmalloc(&den, sizeof(double) * fc) == hipSuccess &&
            dmalloc(&rep_c, sizeof(int) * fc) == hipSuccess &&
            dmalloc(&rep_int, sizeof(int) * fc) == hipSuccess &&
            dmalloc(&bad, sizeof(int)) == hipSuccess &&
            dmalloc(&pw, sizeof(double) * F) == hipSuccess &&
            dmalloc(&pw_perm, sizeof(double) * F) == hipSuccess &&
            dmalloc(&pgram, sizeof(double) * fc) == hipSuccess;
  if (!ok) {
    release();
    drop_new();
    return fail(RR_ERR_DEVICE, "out of device memory for the interpolation weights");
  }
  // eta_k from the operator's passes, prototypes in internal order
  for (int k = 0; k < K; ++k) {
    double* vk = Vi + (size_t)k * F;
    launch_gather(vk, V + (size_t)k * F, h->fperm, F, s);
    launch_csr(h->X, vk, u, nullptr, s);
    Epi e{};
    e.out = t;
    launch_csc(h->X, u, EPI_STORE, e, nullptr, s);
    k_energy<<<1, kBlock, 0, s>>>(F, t, vk, beta, eta + k);
  }
  // coarse features
  bool fine = hipMemsetAsync(bad, 0, sizeof(int), s) == hipSuccess;
  if (rep) {
    fine = fine && hipMemcpyAsync(rep_c, rep, sizeof(int) * fc, hipMemcpyDeviceToDevice, s) == hipSuccess;
  } else {
    k_fill_rep<<<cdiv(fc, kBlock), kBlock, 0, s>>>(fc, rep_c);
    k_rep_min<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, h->labels, h->fperm, rep_c);
  }
  k_rep_internal<<<cdiv(fc, kBlock), kBlock, 0, s>>>(fc, F, rep_c, h->finv, h->labels, rep_int, bad);
  int flag = 0;
  fine = fine && hipMemcpyAsync(&flag, bad, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
  if (!fine || flag) {
    release();
    drop_new();
    return fine ? fail(RR_ERR_INVALID_ARG, "a coarse feature is out of range or outside its cluster")
                : fail(RR_ERR_DEVICE, "interpolation set-up failed on the device");
  }
  k_ls_den<<<cdiv(fc, kBlock), kBlock, 0, s>>>(fc, F, K, Vi, eta, rep_int, den);
  k_ls_weights<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, K, Vi, eta, h->labels, rep_int, den, pw, bad);
  k_perm_vals<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, h->perm, pw, pw_perm);
  {   // diag(P^T P): sum over each cluster of p_j * p_j
    Epi e{};
    e.out = pgram;
    launch_segsum(h->restrict_plan, h->coff + 1, h->perm, pw_perm, pw, EPI_STORE, e, nullptr, s);
  }
  fine = hipMemcpyAsync(&flag, bad, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess && hipGetLastError() == hipSuccess;
  release();
  if (!fine || flag) {
    drop_new();
    return fine ? fail(RR_ERR_INVALID_ARG, "the prototypes give non-finite interpolation weights")
                : fail(RR_ERR_DEVICE, "interpolation set-up failed on the device");
  }
  free_interpolation(h);
  h->lsw = pw;
  h->lsw_perm = pw_perm;
  h->pgram = pgram;
  // the Galerkin coarse Gram P^T X^T X P, one operator application per
  // column; if that fails, the handle goes back to the adjusted square-root
  // average (whose K is rebuilt) rather than keep weights without their K
  rr_status st = build_coarse_gram_valued(h, s);
  if (st != RR_OK) {
    const std::string msg = rr_last_error();
    free_interpolation(h);
    (void)build_coarse_gram(h, s);
    return fail(st, msg);
  }
  if (p_out) launch_gather(p_out, h->lsw, h->finv, F, s);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  return RR_OK;
}

}  // namespace rr
