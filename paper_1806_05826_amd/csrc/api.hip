// C ABI entry points (include/rr.h): handle lifecycle, setup, the PCG driver
// and the step-level calls.  The driver queues whole iterations on the
// caller's stream; all scalars live on the device and kernels skip once the
// device-side `done` flag is set, so the host only polls between chunks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>

#include "rr_device.h"

namespace rr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

rr_status fail(rr_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

__global__ void k_colnorm_binary(int F, const int* col_ptr, double* c) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) c[j] = (double)(col_ptr[j + 1] - col_ptr[j]);
}

// ||x_j||^2 of a valued X: one wave per column (lane-strided sums, fixed
// butterfly), so the long columns of a skewed X take no longer than a wave's
// pass over them
__global__ __launch_bounds__(kBlock) void k_colnorm_values(int F, const int* col_ptr, const double* cval,
                                                           double* c) {
  const int j = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= F) return;
  double s = 0.0;
  for (int e = col_ptr[j] + lane; e < col_ptr[j + 1]; e += 64) s += cval[e] * cval[e];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) c[j] = s;
}

__global__ void k_gather_int(int* dst, const int* src, const int* idx, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

__global__ void k_smooth(int F, const double* r, const double* D, double omega, double* e1) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) e1[j] = (omega * r[j]) / D[j];
}

}  // namespace rr

using namespace rr;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <class T>
rr_status dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = dmalloc((void**)p, sizeof(T) * n);
  if (e != hipSuccess) return fail(RR_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  return RR_OK;
}

void dfree(void* p) {
  if (p) (void)dev_free(p);
}

// A versioned options struct: struct_size bytes of the caller's copy, the
// rest (fields a caller built against an older header lacks) zero, which is
// every field's default.
template <typename T>
rr_status read_opts(const T* in, T* out) {
  *out = T{};
  if (!in) {
    out->struct_size = sizeof(T);
    return RR_OK;
  }
  const uint32_t sz = in->struct_size;
  if (sz < sizeof(uint32_t) || sz > (1u << 16))
    return fail(RR_ERR_INVALID_ARG, "options: struct_size must hold sizeof(the options struct)");
  std::memcpy(out, in, std::min<size_t>(sz, sizeof(T)));
  out->struct_size = sizeof(T);
  return RR_OK;
}

MemCtx* mem_of(const rr_handle* h) { return h ? &const_cast<rr_handle*>(h)->mem : nullptr; }

// A call on a handle living in a caller workspace that ran out of it.
rr_status ws_status(const rr_handle* h, rr_status st) {
  if (st != RR_OK && h && h->mem.mode == MemCtx::kBump && h->mem.overflow)
    return fail(RR_ERR_WORKSPACE, "the handle's workspace is too small (" + std::to_string(h->mem.cap) +
                                      " bytes, " + std::to_string(h->mem.used) + " in use)");
  return st;
}

void free_work(Work& w) {
  dfree(w.x); dfree(w.r); dfree(w.p); dfree(w.q); dfree(w.z); dfree(w.e1); dfree(w.e2);
  dfree(w.rho); dfree(w.b); dfree(w.u); dfree(w.up); dfree(w.c); dfree(w.yc); dfree(w.partials);
  dfree(w.parts.dots);
  dfree(w.sc); dfree(w.D); dfree(w.vin); dfree(w.vout); dfree(w.xref);
  dfree(w.fcg_p); dfree(w.fcg_ap); dfree(w.fcg_paps);
  if (w.sc_host) (void)hipHostFree(w.sc_host);
  IrVectors& f = w.f32;
  dfree(f.x); dfree(f.r); dfree(f.p); dfree(f.q); dfree(f.z); dfree(f.e1); dfree(f.e2);
  dfree(f.D); dfree(f.u); dfree(f.part_cols);
  if (w.extra) {
    dfree(w.X.sell_csc.part);
    dfree(w.X.csc_plan.head); dfree(w.X.csc_plan.tail);
    dfree(w.rplan.head); dfree(w.rplan.tail); dfree(w.rplan.cpart);
    dfree(w.xp_part);
    dfree(w.xr.cpart);
  }
  w.graph.reset();
  if (w.graph.ev) (void)hipEventDestroy(w.graph.ev);
  if (w.stream) (void)hipStreamDestroy(w.stream);
  w = Work{};
}

// The solve vectors and reduction partials of one work set (F features,
// N samples, F_C coarse unknowns, np partials per region).
rr_status alloc_work(Work& w, int F, int N, int FC, int np) {
  RR_TRY(dalloc(&w.x, F)); RR_TRY(dalloc(&w.r, F)); RR_TRY(dalloc(&w.p, F));
  RR_TRY(dalloc(&w.q, F)); RR_TRY(dalloc(&w.z, F)); RR_TRY(dalloc(&w.e1, F));
  RR_TRY(dalloc(&w.e2, F)); RR_TRY(dalloc(&w.rho, F)); RR_TRY(dalloc(&w.b, F));
  RR_TRY(dalloc(&w.D, F)); RR_TRY(dalloc(&w.u, N)); RR_TRY(dalloc(&w.up, N));
  RR_TRY(dalloc(&w.vin, F)); RR_TRY(dalloc(&w.vout, F)); RR_TRY(dalloc(&w.xref, F));
  RR_TRY(dalloc(&w.sc, 1));
  RR_HIP(hipHostMalloc((void**)&w.sc_host, sizeof(Scalars), hipHostMallocDefault));
  std::memset(w.sc_host, 0, sizeof(Scalars));
  if (FC > 0) {
    RR_TRY(dalloc(&w.c, FC));
    RR_TRY(dalloc(&w.yc, FC));
  }
  // five partial regions (pq, upd, rz, init, tr), each large enough for the
  // widest producer grid
  w.npartials = np;
  RR_TRY(dalloc(&w.partials, 5 * (size_t)np));
  w.parts.pq = w.partials;
  w.parts.upd = w.partials + (size_t)np;
  w.parts.rz = w.partials + 2 * (size_t)np;
  w.parts.init = w.partials + 3 * (size_t)np;
  w.parts.tr = w.partials + 4 * (size_t)np;
  w.parts.n_vec = vec_grid(F);
  RR_TRY(dalloc(&w.parts.dots, (size_t)kMaxFcg * kMaxParts));
  return RR_OK;
}

// The flexible-CG ring of a work set: m directions and their images.
rr_status reserve_fcg(Work& w, int m, int F) {
  if (w.fcg_m >= m) return RR_OK;
  dfree(w.fcg_p);
  dfree(w.fcg_ap);
  dfree(w.fcg_paps);
  w.fcg_p = w.fcg_ap = w.fcg_paps = nullptr;
  w.fcg_m = 0;
  RR_TRY(dalloc(&w.fcg_p, (size_t)m * F));
  RR_TRY(dalloc(&w.fcg_ap, (size_t)m * F));
  RR_TRY(dalloc(&w.fcg_paps, kMaxFcg));
  w.fcg_m = m;
  return RR_OK;
}

// Work set k (0: the handle's own); sets beyond the first are created on
// first use with their own partial-sum buffers for the operator passes and
// the restriction.
rr_status get_work_set(rr_handle* h, int k, Work** out) {
  if (k == 0) {
    *out = &h->w;
    return RR_OK;
  }
  while ((int)h->extra_sets.size() < k) {
    Work* w = new (std::nothrow) Work();
    if (!w) return fail(RR_ERR_DEVICE, "out of host memory");
    h->extra_sets.push_back(w);
    w->extra = true;
    w->X = h->X;
    w->rplan = h->restrict_plan;
    w->X.sell_csc.part = nullptr;
    w->X.csc_plan.head = w->X.csc_plan.tail = nullptr;
    w->rplan.head = w->rplan.tail = nullptr;
    w->rplan.cpart = nullptr;
    RR_TRY(alloc_work(*w, h->X.F, h->X.N, h->FC, h->npartials));
    if (h->restrict_plan.ncpart > 0) RR_TRY(dalloc(&w->rplan.cpart, h->restrict_plan.ncpart));
    if (h->X.sliced) RR_TRY(dalloc(&w->X.sell_csc.part, h->X.sell_csc.nout));
    w->xr = h->xp_restrict;
    w->xr.cpart = nullptr;
    if (h->xp.nblk > 0) RR_TRY(dalloc(&w->xp_part, h->xp.nout));
    if (h->xp_restrict.ncpart > 0) RR_TRY(dalloc(&w->xr.cpart, h->xp_restrict.ncpart));
    if (!h->X.binary) {
      RR_TRY(dalloc(&w->X.csc_plan.head, h->X.csc_plan.nblocks));
      RR_TRY(dalloc(&w->X.csc_plan.tail, h->X.csc_plan.nblocks));
    }
    if (h->restrict_plan.nblocks > 0) {
      RR_TRY(dalloc(&w->rplan.head, h->restrict_plan.nblocks));
      RR_TRY(dalloc(&w->rplan.tail, h->restrict_plan.nblocks));
    }
  }
  *out = h->extra_sets[k - 1];
  return RR_OK;
}

void destroy_handle(rr_handle* h) {
  if (!h) return;
  Sparse& X = h->X;
  dfree(X.row_ptr); dfree(X.col_idx); dfree(X.val);
  dfree(X.col_ptr); dfree(X.row_idx); dfree(X.cval);
  free_merge_plan(X.csc_plan);
  free_rows(X.rows);
  free_sell(X.sell_csc);
  free_batch_plan(X.bplan);
  free_merge_plan(h->restrict_plan);
  free_cluster_rows(h->crow);
  free_sell(h->xp);
  free_merge_plan(h->xp_restrict);
  dfree(h->colnorm); dfree(h->gersh); dfree(h->fperm); dfree(h->finv);
  dfree(h->labels); dfree(h->centres); dfree(h->csize); dfree(h->cscale);
  dfree(h->perm); dfree(h->cpos); dfree(h->coff); dfree(h->K);
  for (auto& s : h->slots) { dfree(s.L); dfree(s.Ainv); dfree(s.Dinv); }
  dfree(h->boff); dfree(h->bperm); dfree(h->bgram);
  dfree(h->eig_q); dfree(h->eig_v); dfree(h->rw); dfree(h->wxc);
  free_interpolation(h);
  dfree(h->chol_work); dfree(h->chol_flag); dfree(h->omega_tmp); dfree(h->mlp_scale);
  if (h->pw) {
    dfree(h->pw->v); dfree(h->pw->t); dfree(h->pw->u); dfree(h->pw->D); dfree(h->pw->vin);
    dfree(h->pw->parts); dfree(h->pw->nrm);
    delete h->pw;
  }
  free_mlp(h->mlp);
  dense_free(h);
  free_work(h->w);
  for (Work* w : h->extra_sets) {
    free_work(*w);
    delete w;
  }
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->bstream) (void)hipStreamDestroy(h->bstream);
  delete h;
}

int pick_group(double avg) {
  int g = 4;
  while (g < 64 && g < avg / 2.0) g *= 2;
  return g;
}

rr_status ensure_f32(rr_handle* h, Work& w);   // below: FP32 vectors of refinement
rr_status ensure_power_work(rr_handle* h, int F, int N);   // below

rr_status setup_impl(const rr_csr* Xin, const rr_setup_opts* o, hipStream_t s, rr_handle* h) {
  const double t0 = now_ms();
  RR_HIP(hipGetDevice(&h->device));
  Sparse& X = h->X;
  X.N = (int)Xin->n_rows;
  X.F = (int)Xin->n_cols;
  X.nnz = (int)Xin->nnz;
  X.binary = (Xin->values == nullptr);
  RR_TRY(dalloc(&X.row_ptr, X.N + 1));
  RR_TRY(dalloc(&X.col_idx, X.nnz));
  RR_HIP(hipMemcpyAsync(X.row_ptr, Xin->row_ptr, sizeof(int) * (X.N + 1), hipMemcpyDeviceToDevice, s));
  if (X.nnz)
    RR_HIP(hipMemcpyAsync(X.col_idx, Xin->col_idx, sizeof(int) * X.nnz, hipMemcpyDeviceToDevice, s));
  if (!X.binary) {
    RR_TRY(dalloc(&X.val, X.nnz));
    if (X.nnz) RR_HIP(hipMemcpyAsync(X.val, Xin->values, sizeof(double) * X.nnz, hipMemcpyDeviceToDevice, s));
  }
  rr_status vs = validate_csr(X, s);
  if (vs == RR_ERR_UNSUPPORTED) {
    h->nonneg = false;
  } else if (vs != RR_OK) {
    return vs;
  }
  X.csr_group = pick_group(X.N ? (double)X.nnz / X.N : 1.0);
  RR_TRY(dalloc(&h->fperm, X.F));
  RR_TRY(dalloc(&h->finv, X.F));
  RR_TRY(renumber_features(X, h->fperm, h->finv, s));
  RR_TRY(build_csc(X, s));
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
        ncu > 0)
      X.num_cu = ncu;
  }
  {
    const double tt = now_ms();
    RR_TRY(build_sell_plans(X, s, (o && o->autotune) ? 1 : 0, &h->tuning));
    RR_TRY(build_batch_plan(X.bplan, X, s, (o && o->autotune) ? 1 : 0));
    h->tune_ms = now_ms() - tt;
  }
  // column norms and Gershgorin row sums g = X^T (X 1)
  RR_TRY(dalloc(&h->colnorm, X.F));
  RR_TRY(dalloc(&h->gersh, X.F));
  if (X.binary)
    k_colnorm_binary<<<cdiv(X.F, kBlock), kBlock, 0, s>>>(X.F, X.col_ptr, h->colnorm);
  else
    k_colnorm_values<<<cdiv(X.F, kBlock / 64), kBlock, 0, s>>>(X.F, X.col_ptr, X.cval, h->colnorm);
  // work buffers for the Gershgorin pass (the full set is allocated below)
  Work& w = h->w;
  const int F = X.F, N = X.N;
  RR_TRY(dalloc(&w.x, F));
  RR_TRY(dalloc(&w.u, N));
  RR_TRY(dalloc(&h->omega_tmp, 1));
  {
    launch_fill(w.u, 0.0, N, s);
    launch_fill(w.x, 1.0, F, s);
    launch_csr(X, w.x, w.u, nullptr, s);
    Epi e{};
    e.out = h->gersh;
    // partials are not needed for EPI_STORE
    launch_csc(X, w.u, EPI_STORE, e, nullptr, s);
  }
  // aggregation
  RR_TRY(dalloc(&h->labels, F));
  const int k = o ? o->n_clusters : 0;
  h->k_req = k;
  const double tk = now_ms();
  if (o && o->labels_in) {
    if (o->n_labels_in < 1) return fail(RR_ERR_INVALID_ARG, "n_labels_in must be >= 1");
    RR_TRY(set_labels(h, o->labels_in, o->n_labels_in, s));
  } else if (o && o->lf_tolerance > 0.0) {
    if (!std::isfinite(o->lf_tolerance)) return fail(RR_ERR_INVALID_ARG, "lf_tolerance must be finite");
    int fc = 0;
    RR_TRY(leader_follower(h, o->lf_tolerance, &fc, s));
    h->n_centres = fc;
    RR_TRY(set_labels(h, nullptr, fc, s));
  } else if (k > 0) {
    RR_TRY(dalloc(&h->centres, std::min(k, F)));
    const int mi = (o->kmeans_max_iter > 0) ? o->kmeans_max_iter : 100;
    RR_TRY(run_kmeans(h, k, o->seed, mi, s));
  }
  h->kmeans_ms = now_ms() - tk;
  int np = cdiv(F, kBlock) + 1;   // >= every reduction grid (the segment reduction uses <= 256)
  if (!X.binary) np = std::max(np, X.csc_plan.nblocks + cdiv(X.csc_plan.nspan, kBlock / 64) + 1);
  if (h->FC > 0 && X.binary) RR_TRY(check_coarse_size(h->FC));   // before the F_C^2 buffers
  if (h->FC > 0) {
    const int fc = h->FC;
    RR_TRY(dalloc(&h->K, (size_t)fc * fc));
    RR_TRY(build_coarse_gram(h, s));
    const int nslots = (o && o->lambda_slots > 0) ? o->lambda_slots : 4;
    h->slots.resize(nslots);
    for (auto& sl : h->slots) {
      RR_TRY(dalloc(&sl.L, (size_t)fc * fc));
      RR_TRY(dalloc(&sl.Ainv, (size_t)fc * fc));
    }
    RR_TRY(dalloc(&h->chol_work, 2 * (size_t)fc * fc));
    RR_TRY(dalloc(&h->chol_flag, 1));
    if (o && o->block_smoother) RR_TRY(build_smoother_blocks(h, s));
    RR_TRY(build_cluster_rows(h, s));
    if (o && o->coarse_eigen) RR_TRY(coarse_eigen(h, &h->eig_sweeps, s));
    np = std::max(np, h->restrict_plan.nblocks + cdiv(h->restrict_plan.nspan, kBlock / 64) + 1);
  }
  np = std::max(np, std::max(3 * kMaxParts, kMaxReduceBlocks + 1));
  h->npartials = np;
  RR_HIP(hipStreamSynchronize(s));
  dfree(w.x);
  dfree(w.u);
  w.x = w.u = nullptr;
  RR_TRY(alloc_work(w, F, N, h->FC, np));
  RR_HIP(hipMemsetAsync(w.sc, 0, sizeof(Scalars), s));
  w.X = h->X;
  w.rplan = h->restrict_plan;
  w.xp_part = h->xp.part;
  w.xr = h->xp_restrict;
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  // buffers of later solves, reserved now so that those solves allocate
  // nothing: the power-iteration vectors (X with negative entries, the block
  // smoother's weight), the block smoother's inverses of every lambda slot
  if (!h->nonneg || h->nblk > 0) RR_TRY(ensure_power_work(h, F, N));
  for (auto& sl : h->slots)
    if (h->nblk > 0 && !sl.Dinv) RR_TRY(dalloc(&sl.Dinv, (size_t)h->nblk * 32 * 32));
  if (o && o->reserve_fcg_m > 0) RR_TRY(reserve_fcg(h->w, std::min(o->reserve_fcg_m, kMaxFcg), X.F));
  if (o && o->reserve_sets > 0) {
    if (o->reserve_sets > 64) return fail(RR_ERR_INVALID_ARG, "reserve_sets must be <= 64");
    for (int k = 1; k <= o->reserve_sets; ++k) {
      Work* w = nullptr;
      RR_TRY(get_work_set(h, k, &w));
      if (o->reserve_fcg_m > 0) RR_TRY(reserve_fcg(*w, std::min(o->reserve_fcg_m, kMaxFcg), X.F));
    }
  }
  if (o && o->reserve_f32 && X.binary) RR_TRY(ensure_f32(h, h->w));
  h->setup_ms = now_ms() - t0;
  return RR_OK;
}

rr_status check_handle(const rr_handle* h) {
  if (!h) return fail(RR_ERR_INVALID_ARG, "null handle");
  return RR_OK;
}

// Calls built on the sparse operator.
rr_status check_sparse(const rr_handle* h) {
  RR_TRY(check_handle(h));
  if (h->dense)
    return fail(RR_ERR_UNSUPPORTED, "not available for a dense handle (use rr_solve_block, "
                                    "rr_apply_operator_block)");
  return RR_OK;
}

rr_status check_lambda(double lam, bool allow_zero) {
  if (!std::isfinite(lam) || lam < 0.0 || (!allow_zero && lam == 0.0))
    return fail(RR_ERR_INVALID_ARG, "lambda must be finite and > 0");
  return RR_OK;
}

// ---- smoother weight by power iteration (X with negative entries) ---------

// v = s * v / rho (rho = *nrm, or 1 before the first product); s = D^-1/2
__global__ void k_pw_scale(int F, const double* __restrict__ v, const double* __restrict__ D,
                           const double* nrm, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) out[j] = v[j] / (sqrt(D[j]) * (nrm ? *nrm : 1.0));
}

// w = s * t and the block partials of ||w||^2
__global__ __launch_bounds__(kBlock) void k_pw_post(int F, const double* __restrict__ t,
                                                    const double* __restrict__ D,
                                                    double* __restrict__ w, double* parts) {
  double acc = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) {
    const double x = t[j] / sqrt(D[j]);
    w[j] = x;
    acc += x * x;
  }
  __shared__ double red[kBlock / 64];
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) parts[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_pw_norm(const double* parts, int n, double* nrm) {
  __shared__ double red[kBlock / 64];
  const double t = sum_parts<kBlock>(parts, n, red);
  if (threadIdx.x == 0) *nrm = sqrt(t);
}

// Buffers of the power-iteration smoother weight (X with negative entries,
// and the block smoother's weight).
rr_status ensure_power_work(rr_handle* h, int F, int N) {
  if (h->pw) return RR_OK;
  h->pw = new (std::nothrow) rr_handle::PowerWork();
  if (!h->pw) return fail(RR_ERR_DEVICE, "out of host memory");
  RR_TRY(dalloc(&h->pw->v, F)); RR_TRY(dalloc(&h->pw->t, F)); RR_TRY(dalloc(&h->pw->u, N));
  RR_TRY(dalloc(&h->pw->D, F)); RR_TRY(dalloc(&h->pw->vin, F));
  RR_TRY(dalloc(&h->pw->parts, kMaxParts)); RR_TRY(dalloc(&h->pw->nrm, 1));
  return RR_OK;
}

// The oracle's power estimate: 30 products with D^-1/2 A D^-1/2 from a
// start vector with SplitMix64(kPowerSeed) entries in [0.5, 1.5) (caller's
// feature order), rho = the last norm ratio, omega = 1 / (1.1 rho).
constexpr uint64_t kPowerSeed = 0x5eedULL;
rr_status omega_power(rr_handle* h, const Sparse& X, double lam, double* omega, hipStream_t s) {
  const int F = X.F, N = X.N;
  RR_TRY(ensure_power_work(h, F, N));
  rr_handle::PowerWork& p = *h->pw;
  std::vector<double> v0(F);
  uint64_t st = kPowerSeed;
  double ss = 0.0;
  for (int j = 0; j < F; ++j) {
    v0[j] = (double)(splitmix64_next(st) >> 11) * (1.0 / 9007199254740992.0) + 0.5;
    ss += v0[j] * v0[j];
  }
  const double inv = 1.0 / std::sqrt(ss);
  for (auto& x : v0) x *= inv;
  RR_HIP(hipMemcpyAsync(p.vin, v0.data(), sizeof(double) * F, hipMemcpyHostToDevice, s));
  launch_gather(p.v, p.vin, h->fperm, F, s);   // caller order -> internal order
  launch_colnorm_diag(F, h->colnorm, lam, p.D, s);
  const int g = vec_grid(F);
  for (int it = 0; it < 30; ++it) {
    // t = A (s v / rho); v = s t
    k_pw_scale<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, p.v, p.D, it ? p.nrm : nullptr, p.vin);
    if (h->dense) {
      RR_TRY(dense_apply_one(h, p.vin, lam, p.t, s));
    } else {
      launch_csr(X, p.vin, p.u, nullptr, s);
      Epi e{};
      e.lam = lam;
      e.p = p.vin;
      e.out = p.t;
      launch_csc(X, p.u, EPI_APPLY, e, nullptr, s);
    }
    k_pw_post<<<g, kBlock, 0, s>>>(F, p.t, p.D, p.v, p.parts);
    k_pw_norm<<<1, kBlock, 0, s>>>(p.parts, g, p.nrm);
  }
  double rho = 0.0;
  RR_HIP(hipMemcpyAsync(&rho, p.nrm, sizeof(double), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(RR_ERR_BREAKDOWN, "power iteration failed");
  *omega = 1.0 / (1.1 * rho);
  return RR_OK;
}

// X is the operator view of the work set whose stream s runs the estimate:
// its partial-sum buffers are ordered with that set's own solve.
__global__ void k_div_by(int F, const double* __restrict__ v, const double* nrm, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) out[j] = v[j] / *nrm;
}

__global__ __launch_bounds__(kBlock) void k_sq_parts(int F, const double* __restrict__ v, double* parts) {
  double acc = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < F; j += gridDim.x * kBlock) acc += v[j] * v[j];
  __shared__ double red[kBlock / 64];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) parts[blockIdx.x] = t;
}

// The block smoother's weight: 30 power steps v <- D_B^-1 A v / ||.|| from
// the same start vector as omega_power; omega = 1 / (1.1 rho).
rr_status omega_block_power(rr_handle* h, const Sparse& X, double lam, LambdaSlot& sl, hipStream_t s) {
  const int F = X.F, N = X.N;
  RR_TRY(ensure_power_work(h, F, N));
  rr_handle::PowerWork& p = *h->pw;
  std::vector<double> v0(F);
  uint64_t st = kPowerSeed;
  double ss = 0.0;
  for (int j = 0; j < F; ++j) {
    v0[j] = (double)(splitmix64_next(st) >> 11) * (1.0 / 9007199254740992.0) + 0.5;
    ss += v0[j] * v0[j];
  }
  const double inv = 1.0 / std::sqrt(ss);
  for (auto& x : v0) x *= inv;
  RR_HIP(hipMemcpyAsync(p.v, v0.data(), sizeof(double) * F, hipMemcpyHostToDevice, s));
  launch_gather(p.vin, p.v, h->fperm, F, s);   // caller order -> internal order
  const int g = vec_grid(F);
  for (int it = 0; it < 30; ++it) {
    if (it) k_div_by<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, p.v, p.nrm, p.vin);
    launch_csr(X, p.vin, p.u, nullptr, s);
    Epi e{};
    e.lam = lam;
    e.p = p.vin;
    e.out = p.t;
    launch_csc(X, p.u, EPI_APPLY, e, nullptr, s);
    launch_block_smooth(h, sl.Dinv, 1.0, p.t, nullptr, nullptr, nullptr, p.v, nullptr, nullptr, s);
    k_sq_parts<<<g, kBlock, 0, s>>>(F, p.v, p.parts);
    k_pw_norm<<<1, kBlock, 0, s>>>(p.parts, g, p.nrm);
  }
  double rho = 0.0;
  RR_HIP(hipMemcpyAsync(&rho, p.nrm, sizeof(double), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(RR_ERR_BREAKDOWN, "block power iteration failed");
  sl.omega_block = 1.0 / (1.1 * rho);
  return RR_OK;
}

rr_status auto_omega(rr_handle* h, const Sparse& X, double lam, double* omega, hipStream_t s) {
  if (!h->nonneg) return omega_power(h, X, lam, omega, s);
  launch_omega_gersh(h->X.F, h->gersh, h->colnorm, lam, h->omega_tmp, nullptr, nullptr, s);
  RR_HIP(hipMemcpyAsync(omega, h->omega_tmp, sizeof(double), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  return RR_OK;
}

// The coarse factor for lambda, from the cache or freshly computed.
rr_status get_slot(rr_handle* h, const Sparse& X, double lam, LambdaSlot** out, double* ms, hipStream_t s) {
  *ms = 0.0;
  for (auto& sl : h->slots)
    if (sl.valid && sl.lam == lam) {
      sl.stamp = ++h->stamp;
      *out = &sl;
      return RR_OK;
    }
  LambdaSlot* victim = nullptr;
  for (auto& sl : h->slots)
    if (sl.in_use == 0 && (!victim || !sl.valid || (victim->valid && sl.stamp < victim->stamp)))
      victim = &sl;
  if (!victim) {   // every cached factor is in use by a running solve
    LambdaSlot ns;
    const int fc = h->FC;
    RR_TRY(dalloc(&ns.L, (size_t)fc * fc));
    RR_TRY(dalloc(&ns.Ainv, (size_t)fc * fc));
    h->slots.push_back(ns);   // slots is a deque: pointers to other slots stay valid
    victim = &h->slots.back();
  }
  const double t0 = now_ms();
  victim->valid = false;
  RR_TRY(h->eig_q ? coarse_from_eigen(h, lam, *victim, s) : coarse_factor(h, lam, *victim, s));
  RR_TRY(block_factor(h, lam, *victim, s));
  RR_TRY(auto_omega(h, X, lam, &victim->omega, s));
  RR_HIP(hipStreamSynchronize(s));
  victim->lam = lam;
  victim->valid = true;
  victim->stamp = ++h->stamp;
  *out = victim;
  *ms = now_ms() - t0;
  return RR_OK;
}

struct Prof {
  bool on = false;
  std::vector<std::pair<int, int>> csr, csc;   // event-triple index, iteration tag
  int used = 0;
};

// Three events per timed pass: start, after the gather kernel, end.
rr_status prof_pair(rr_handle* h, Prof& pf, int* idx) {
  const int need = 3 * (pf.used + 1);
  while ((int)h->ev_pool.size() < need) {
    hipEvent_t e;
    RR_HIP(hipEventCreate(&e));
    h->ev_pool.push_back(e);
  }
  *idx = pf.used++;
  return RR_OK;
}

// Apply the operator pieces with optional event timing.
// With pu, v holds z and the pass forms w.up = X z + beta w.up, X p of the
// new direction (the column pass after it reads w.up and uses
// EPI_APPLY_DOT_P).  Without, the pass writes uout (w.u by default).
rr_status op_csr(rr_handle* h, Work& w, Prof& pf, int tag, const double* v, hipStream_t s,
                 const StageArgs* stage = nullptr, const PUpd* pu = nullptr, double* uout = nullptr) {
  const int* done = &w.sc->done;
  double* u = uout ? uout : w.u;
  if (!pf.on) {
    if (pu)
      launch_csr_pupd(w.X, v, w.up, done, s, *pu);
    else
      launch_csr(w.X, v, u, done, s, stage);
    return RR_OK;
  }
  int i;
  RR_TRY(prof_pair(h, pf, &i));
  RR_HIP(hipEventRecord(h->ev_pool[3 * i], s));
  if (pu)
    launch_csr_pupd(w.X, v, w.up, done, s, *pu, h->ev_pool[3 * i + 1]);
  else
    launch_csr(w.X, v, u, done, s, stage, h->ev_pool[3 * i + 1]);
  RR_HIP(hipEventRecord(h->ev_pool[3 * i + 2], s));
  pf.csr.push_back({i, tag});
  return RR_OK;
}

// *nparts receives the count of block partials a dot-product epilogue left.
rr_status op_csc(rr_handle* h, Work& w, Prof& pf, int tag, int mode, const Epi& e, hipStream_t s,
                 int* nparts = nullptr, const double* uin = nullptr) {
  const int* done = &w.sc->done;
  const double* u = uin ? uin : w.u;
  if (!pf.on) {
    const int n = launch_csc(w.X, u, mode, e, done, s);
    if (nparts) *nparts = n;
    return RR_OK;
  }
  int i;
  RR_TRY(prof_pair(h, pf, &i));
  RR_HIP(hipEventRecord(h->ev_pool[3 * i], s));
  const int n = launch_csc(w.X, u, mode, e, done, s, h->ev_pool[3 * i + 1]);
  if (nparts) *nparts = n;
  RR_HIP(hipEventRecord(h->ev_pool[3 * i + 2], s));
  pf.csc.push_back({i, tag});
  return RR_OK;
}

Epi base_epi(const Work& w, double lam) {
  Epi e{};
  e.lam = lam;
  e.sc = w.sc;
  e.D = w.D;
  return e;
}

// z = B r for the two-level forms; e1 (V-cycle) must already hold w D^-1 r.
// The partials of <r, z> are left in parts.rz (*n_rz of them).  With a
// stage, the convergence check of the preceding update runs first.
rr_status precond_two_level(rr_handle* h, Work& w, Prof& pf, int tag, int kind, double lam,
                            double omega, const LambdaSlot& sl, const double* r, double* z,
                            const StageArgs* stage, int* n_rz, hipStream_t s,
                            double* snap = nullptr) {
  const int F = h->X.F;
  const int* done = &w.sc->done;
  if (kind == PK_ROUGHER) {
    // e1 = rsteps CG steps on A e = r from 0, rho its residual; then
    // z = e1 + P A_c^-1 P^T rho (pre-smoothing only, as in the paper's runs)
    double* rr_a = w.parts.init;
    double* rr_b = w.parts.tr;
    const int nv = w.parts.n_vec;
    const double* Dj = w.rjacobi ? w.D : nullptr;
    launch_rg_start(F, r, Dj, w.e2, rr_a, w.sc, stage, s);
    for (int i = 0; i < w.rsteps; ++i) {
      RR_TRY(op_csr(h, w, pf, tag, w.e2, s));
      Epi eq = base_epi(w, lam);
      eq.p = w.e2;
      eq.out = w.q;
      eq.partials = w.parts.pq;
      int npq = 0;
      RR_TRY(op_csc(h, w, pf, tag, EPI_APPLY_DOT, eq, s, &npq));
      launch_rg_step(F, i == 0, r, Dj, w.e1, w.rho, w.e2, w.q, rr_a, nv, w.parts.pq, npq, rr_b, w.sc,
                     s);
      if (i + 1 < w.rsteps) launch_rg_dir(F, w.rho, Dj, w.e2, rr_b, nv, rr_a, nv, w.sc, s);
      std::swap(rr_a, rr_b);
    }
    launch_restrict(h, w.rplan, w.rho, w.c, done, s);
    launch_gemv(h->FC, sl.Ainv, w.c, w.yc, done, s);
    launch_prolong(F, h->labels, h->cscale, w.yc, w.e1, z, nullptr, nullptr, 0.0, 0, w.sc, nullptr, s,
                   h->lsw);
    *n_rz = 0;
    return RR_OK;
  }
  if (kind == PK_ADDITIVE) {
    if (stage) launch_stage_update(*stage, s);
    launch_restrict(h, w.rplan, r, w.c, done, s);
    launch_gemv(h->FC, sl.Ainv, w.c, w.yc, done, s);
    if (w.block) {   // z = w D_B^-1 r + P yc
      *n_rz = launch_block_smooth(h, sl.Dinv, omega, r, nullptr, w.yc, r, z, w.parts.rz, done, s);
      return RR_OK;
    }
    launch_prolong(F, h->labels, h->cscale, w.yc, nullptr, z, r, w.D, omega, 1, w.sc,
                   w.parts.rz, s, h->lsw);
    *n_rz = w.parts.n_vec;
    return RR_OK;
  }
  // block smoother: e1 = w D_B^-1 r replaces the point step the update formed
  // (on the iteration that converges this is wasted work, nothing more)
  if (w.block)
    launch_block_smooth(h, sl.Dinv, omega, r, nullptr, nullptr, nullptr, w.e1, nullptr, done, s);
  const bool label_rows = h->crow.nlayer > 0 && !h->lsw;
  if (kind == PK_VCYCLE && label_rows && !w.block && !snap && h->X.binary && h->xp.nblk > 0 && w.xp_part &&
      (w.xr.ncpart == 0 || w.xr.cpart) && restrict_gemv_fusable(w.xr, h->FC)) {
    // P^T (r - A e1) = P^T (r - lam e1) - (X P)^T (X e1): the row pass's u
    // goes straight to the column pass of X P (F_C segments), so the residual
    // r - A e1 is never formed at the fine level
    RR_TRY(op_csr(h, w, pf, tag, w.e1, s, stage));
    SellPlan xp = h->xp;
    xp.part = w.xp_part;
    launch_sell_gather(xp, w.u, s, done);
    launch_restrict_gemv_xp(w.xr, h->perm, r, w.e1, lam, h->cscale, xp, w.xp_part, w.c, h->FC, sl.Ainv, w.yc,
                            done, s);
    launch_cluster_rows(h, w.yc, w.X.rw, w.u, done, s);
    Epi ep = base_epi(w, lam);
    ep.p = w.e1;
    ep.r = r;
    ep.omega = omega;
    ep.out = z;
    ep.partials = w.parts.rz;
    ep.labels = h->labels;
    ep.cscale = h->cscale;
    ep.yc = w.yc;
    RR_TRY(op_csc(h, w, pf, tag, EPI_POST_P, ep, s, n_rz));
    return RR_OK;
  }
  // V(1,1): rho1 = r - A e1
  RR_TRY(op_csr(h, w, pf, tag, w.e1, s, stage));
  Epi e = base_epi(w, lam);
  e.p = w.e1;
  e.r = r;
  e.out = w.rho;
  e.opos = h->cpos;   // rho1 in cluster order: the restriction reads it contiguously
  RR_TRY(op_csc(h, w, pf, tag, EPI_RESID, e, s));
  // e2 = e1 + P A_c^-1 P^T rho1 (learned: the network's coarse correction)
  if (kind != PK_LEARNED && !snap && restrict_gemv_fusable(w.rplan, h->FC)) {
    launch_restrict_gemv(w.rplan, w.rho, h->lsw ? h->lsw_perm : nullptr, h->lsw ? nullptr : h->cscale, w.c,
                         h->FC, sl.Ainv, w.yc, done, s);
  } else {
    launch_restrict_sorted(h, w.rplan, w.rho, w.c, done, s);
  }
  if (snap) launch_copy_done(snap, w.c, h->FC, done, s);
  if (kind == PK_LEARNED) {
    launch_learned_in(h->FC, w.c, lam, h->mlp.xb, h->mlp_scale, done, s);
    mlp_forward(h->mlp, 1, s);
    launch_learned_out(h->FC, h->mlp.y, h->mlp_scale, h->K, lam, w.yc, done, s);
  } else if (snap || !restrict_gemv_fusable(w.rplan, h->FC)) {
    launch_gemv(h->FC, sl.Ainv, w.c, w.yc, done, s);
  }
  // z = e2 + w D^-1 (r - A e2), <r,z> -> beta; X e2 = X e1 + X P yc, where
  // u still holds X e1 (the label table carries the square-root-average P).
  // With the point smoother, e2 = e1 + P yc is formed inside the column
  // pass's epilogue, the only place that reads it.
  if (label_rows && !w.block && h->X.binary) {
    launch_cluster_rows(h, w.yc, w.X.rw, w.u, done, s);
    Epi ep = base_epi(w, lam);
    ep.p = w.e1;
    ep.r = r;
    ep.omega = omega;
    ep.out = z;
    ep.partials = w.parts.rz;
    ep.labels = h->labels;
    ep.cscale = h->cscale;
    ep.yc = w.yc;
    RR_TRY(op_csc(h, w, pf, tag, EPI_POST_P, ep, s, n_rz));
    return RR_OK;
  }
  launch_prolong(F, h->labels, h->cscale, w.yc, w.e1, w.e2, nullptr, nullptr, 0.0, 0, w.sc, nullptr, s,
                 h->lsw);
  if (label_rows)
    launch_cluster_rows(h, w.yc, w.X.rw, w.u, done, s);
  else
    RR_TRY(op_csr(h, w, pf, tag, w.e2, s));
  if (w.block) {   // rho2 = r - A e2, then z = e2 + w D_B^-1 rho2
    Epi eb = base_epi(w, lam);
    eb.p = w.e2;
    eb.r = r;
    eb.out = w.rho;
    RR_TRY(op_csc(h, w, pf, tag, EPI_RESID, eb, s));
    *n_rz = launch_block_smooth(h, sl.Dinv, omega, w.rho, w.e2, nullptr, r, z, w.parts.rz, done, s);
    return RR_OK;
  }
  Epi e2 = base_epi(w, lam);
  e2.p = w.e2;
  e2.r = r;
  e2.omega = omega;
  e2.out = z;
  e2.partials = w.parts.rz;
  RR_TRY(op_csc(h, w, pf, tag, EPI_POST, e2, s, n_rz));
  return RR_OK;
}

// One solve, in phases so that several solves (distinct handles) can be
// queued round-robin on their own streams: begin (checks, b, init, first
// preconditioner application), queue_chunk (a chunk of iterations), poll
// (read the device scalars), finish (w, the true residual, info).
struct Solve {
  rr_handle* h = nullptr;
  Work* ws = nullptr;      // the work set this solve runs in
  double lam = 0.0;
  const double* rhs = nullptr;
  double* wout = nullptr;
  rr_solve_opts op{};
  hipStream_t s = nullptr;
  double t0 = 0.0, coarse_ms = 0.0, omega = 0.0;
  int kind = 0, chunk = 8, fcg_m = 1, queued = 0;
  bool two_level = false, done = false;
  LambdaSlot* sl = nullptr;
  const double* xref = nullptr;
  StageArgs stage{};
  Prof pf;
  // coarse residual snapshots P^T r_k after every `snap_every`-th update
  double* snap = nullptr;
  int snap_every = 0, snap_max = 0, snap_queued = 0;
  // learned coarse correction: switch to the algebraic cycle on a stall or
  // on a failed step (the flexible-CG history then restarts at fcg_base)
  double last_rr = -1.0;
  int fallback_iter = -1;
  int fcg_base = 0;
  bool skip_check = false;   // no update since the last convergence check
  // PCG with a two-level preconditioner: the direction update p = z + beta p
  // is left to the next iteration (pu_pending): its row pass forms
  // X p = X z + beta X p from the previous direction's X p, and its column
  // reduction writes p; beta's partials are the preconditioner's <r,z>
  // partials (pu_n of them)
  bool pu_fold = false, pu_pending = false;
  int pu_n = 0;
  // precision RR_PREC_F32_CYCLE: the preconditioner's cycle runs in FP32
  bool cycle32 = false;
  // continuation of a PCG solve left by the persistent kernel: the work set
  // holds b, x, r and p of iteration `iter`, whose <r,z> is rz
  struct Resume {
    int iter;
    double rz, bb, rr;
  };
  const Resume* resume = nullptr;
  rr_status precond(int tag, const StageArgs* st, int* nrz, double* snap_to = nullptr);

  rr_status begin();
  rr_status queue_chunk();
  rr_status queue_chunk_eager(Work& w, int F);
  rr_status poll();
  rr_status finish(rr_solve_info* info);
  void release() {
    if (sl) sl->in_use--;
    sl = nullptr;
  }
};

rr_status precond32(rr_handle* h, Work& w, double lam, double omega, const LambdaSlot& sl,
                    const StageArgs* stage, int* n_rz, hipStream_t s);   // below

// z = B r with the solve's preconditioner (two-level forms), in FP64 or as
// the FP32 cycle whose z is widened back.
rr_status Solve::precond(int tag, const StageArgs* st, int* nrz, double* snap_to) {
  Work& w = *ws;
  if (cycle32) {
    const int F = h->X.F;
    const int* done = &w.sc->done;
    launch_cycle_in(F, w.r, h->colnorm, lam, omega, w.f32, done, s);
    RR_TRY(precond32(h, w, lam, omega, *sl, st, nrz, s));
    launch_widen(F, w.f32.z, w.z, done, s);
    return RR_OK;
  }
  return precond_two_level(h, w, pf, tag, kind, lam, omega, *sl, w.r, w.z, st, nrz, s, snap_to);
}

rr_status Solve::begin() {
  t0 = now_ms();
  RR_TRY(check_lambda(lam, false));
  if (!rhs || !wout) return fail(RR_ERR_INVALID_ARG, "null rhs or w");
  kind = op.precond;
  if (kind < 0 || kind > 5) return fail(RR_ERR_INVALID_ARG, "unknown preconditioner");
  if ((kind == PK_VCYCLE || kind == PK_ADDITIVE || kind == PK_LEARNED || kind == PK_ROUGHER) &&
      h->FC == 0)
    return fail(RR_ERR_INVALID_ARG, "two-level preconditioner needs a coarse level (n_clusters > 0)");
  if (kind == PK_ROUGHER) {
    if (op.krylov != RR_KRYLOV_FCG)
      return fail(RR_ERR_INVALID_ARG, "the CG rougher is nonlinear: use flexible CG");
    if (op.rougher_steps < 0 || op.rougher_steps > 16)
      return fail(RR_ERR_INVALID_ARG, "rougher_steps must be in [0, 16]");
  }
  ws->rsteps = op.rougher_steps > 0 ? op.rougher_steps : 2;
  ws->rjacobi = op.rougher_jacobi != 0;
  if (kind == PK_LEARNED) {
    if (op.krylov != RR_KRYLOV_FCG)
      return fail(RR_ERR_INVALID_ARG, "the learned coarse correction is nonlinear: use flexible CG");
    if (!h->mlp.w || h->mlp.in != h->FC + 1 || h->mlp.out != h->FC)
      return fail(RR_ERR_INVALID_ARG, "no network for this coarse level (rr_mlp_init)");
  }
  if (op.fixed_iters < 0 || op.max_iter < 0 || op.chunk < 0 || op.tol < 0 || op.err_tol < 0)
    return fail(RR_ERR_INVALID_ARG, "negative option");
  if (op.krylov != RR_KRYLOV_PCG && op.krylov != RR_KRYLOV_FCG)
    return fail(RR_ERR_INVALID_ARG, "unknown Krylov method");
  if (op.fcg_m < 0 || op.fcg_m > kMaxFcg)
    return fail(RR_ERR_INVALID_ARG, "fcg_m must be in [0, 16]");
  const double tol = op.tol > 0 ? op.tol : 1e-10;
  const int max_iter = op.max_iter > 0 ? op.max_iter : 10000;
  chunk = op.chunk > 0 ? op.chunk : 8;
  Work& w = *ws;
  const int F = h->X.F;
  fcg_m = op.fcg_m > 0 ? op.fcg_m : 1;
  if (op.krylov == RR_KRYLOV_FCG && w.fcg_m < fcg_m) {
    RR_HIP(hipStreamSynchronize(s));
    RR_TRY(reserve_fcg(w, fcg_m, F));
  }
  if (op.smoother != RR_SMOOTHER_POINT && op.smoother != RR_SMOOTHER_BLOCK)
    return fail(RR_ERR_INVALID_ARG, "unknown smoother");
  const bool block = op.smoother == RR_SMOOTHER_BLOCK;
  if (block && !(kind == PK_VCYCLE || kind == PK_ADDITIVE || kind == PK_LEARNED))
    return fail(RR_ERR_INVALID_ARG, "the block smoother belongs to the two-level forms");
  if (block && h->nblk == 0)
    return fail(RR_ERR_INVALID_ARG, "no smoother blocks: set up with block_smoother = 1");
  if (block && w.X.rw) return fail(RR_ERR_UNSUPPORTED, "the block smoother is built for unweighted X");
  if (h->lsw && (block || kind == PK_LEARNED))
    return fail(RR_ERR_UNSUPPORTED,
                "least-squares interpolation is built for the point smoother and the algebraic coarse solve");
  w.block = block;
  cycle32 = op.precision == RR_PREC_F32_CYCLE;
  if (cycle32) {
    if (kind != PK_VCYCLE || op.krylov != RR_KRYLOV_FCG)
      return fail(RR_ERR_INVALID_ARG, "the FP32 cycle runs the V(1,1) preconditioner under flexible CG");
    if (!h->X.binary || w.X.rw || h->lsw || block)
      return fail(RR_ERR_UNSUPPORTED, "the FP32 cycle is built for unweighted 0/1 X with the point "
                                      "smoother and the square-root-average P");
    RR_TRY(ensure_f32(h, w));
  }
  omega = op.omega;
  if (kind == PK_VCYCLE || kind == PK_ADDITIVE || kind == PK_LEARNED || kind == PK_ROUGHER) {
    RR_TRY(get_slot(h, w.X, lam, &sl, &coarse_ms, s));
    sl->in_use++;
    if (block && sl->omega_block == 0.0) RR_TRY(omega_block_power(h, w.X, lam, *sl, s));
    if (omega == 0.0) omega = block ? sl->omega_block : sl->omega;
  }
  if (!std::isfinite(omega) || omega < 0.0) return fail(RR_ERR_INVALID_ARG, "omega must be finite and >= 0");
  launch_colnorm_diag(F, h->colnorm, lam, w.D, s);
  if (resume) {
    // the next iteration's update takes alpha = rz / <p, A p> and forms e1
    // from the new r itself; the convergence checks resume at the first update
    if (op.krylov != RR_KRYLOV_PCG || (kind != PK_VCYCLE && kind != PK_JACOBI) || op.x_ref ||
        op.residual_history || block || w.X.rw)
      return fail(RR_ERR_INVALID_ARG, "internal: only FP64 PCG solves with V(1,1) or Jacobi continue");
    Scalars& hs = *w.sc_host;
    std::memset(&hs, 0, sizeof(Scalars));
    hs.bb = resume->bb;
    hs.tol2 = tol * tol * resume->bb;
    hs.limit = op.fixed_iters > 0 ? op.fixed_iters : max_iter;
    hs.fixed = op.fixed_iters;
    hs.status = RR_ERR_NOT_CONVERGED;
    hs.rz = hs.rz_next = resume->rz;
    hs.rr = resume->rr;
    hs.iter = resume->iter;
    RR_HIP(hipMemcpyAsync(w.sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, s));
    pf.on = false;
    two_level = kind == PK_VCYCLE;
    stage = StageArgs{w.sc, w.parts.upd, w.parts.n_vec, nullptr, kind};
    queued = resume->iter;
    // p is ready: the first iteration applies A to it and keeps X p, the
    // later ones fold their direction updates
    pu_fold = two_level && csr_pupd_ok(w.X);
    pu_pending = false;
    return RR_OK;
  }
  if (op.rhs_is_b) {
    launch_gather(w.b, rhs, h->fperm, F, s);
  } else {
    Epi e{};
    e.out = w.b;
    if (w.X.rw) {   // weighted least squares: b = X^T D y
      launch_row_scale(w.X.N, w.X.rw, rhs, w.u, s);
      launch_csc(w.X, w.u, EPI_STORE, e, nullptr, s);
    } else {
      launch_csc(w.X, rhs, EPI_STORE, e, nullptr, s);
    }
  }
  Scalars& hs = *w.sc_host;
  std::memset(&hs, 0, sizeof(Scalars));
  hs.tol2 = tol * tol;
  hs.errtol2 = op.err_tol * op.err_tol;
  hs.limit = op.fixed_iters > 0 ? op.fixed_iters : max_iter;
  hs.fixed = op.fixed_iters;
  hs.use_err = (op.x_ref != nullptr) ? 1 : 0;
  hs.status = RR_ERR_NOT_CONVERGED;
  RR_HIP(hipMemcpyAsync(w.sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, s));
  pf.on = op.profile != 0;
  if (op.x_ref) {
    launch_gather(w.xref, op.x_ref, h->fperm, F, s);
    xref = w.xref;
  }
  two_level = (kind == PK_VCYCLE || kind == PK_ADDITIVE || kind == PK_LEARNED || kind == PK_ROUGHER);
  const int nv = w.parts.n_vec;
  launch_pcg_init(F, w.b, w.x, w.r, w.p, w.z, w.e1, w.D, xref, omega, kind, w.parts.init, s);
  launch_finish_init(w.sc, w.parts.init, nv, op.residual_history, kind, s);
  // the convergence check after each update runs in the kernel that follows it
  stage = StageArgs{w.sc, w.parts.upd, nv, op.residual_history, kind};
  queued = 0;
  if (op.krylov == RR_KRYLOV_FCG) {
    if (two_level) {
      int nrz = 0;
      RR_TRY(precond(-1, nullptr, &nrz));
    }
  } else if (two_level) {
    int nrz = 0;
    RR_TRY(precond_two_level(h, w, pf, -1, kind, lam, omega, *sl, w.r, w.z, nullptr, &nrz, s));
    // the first direction p = z: sc->rz is still 0, so the folded update
    // takes beta = 0
    pu_fold = csr_pupd_ok(w.X);
    if (pu_fold) {
      pu_pending = true;
      pu_n = nrz;
    } else {
      launch_pupdate(F, w.p, w.z, w.sc, w.parts.rz, nrz, 1, nullptr, s);
    }
  } else {
    launch_pupdate(F, w.p, w.z, w.sc, w.parts.init + 2 * nv, nv, 1, nullptr, s);
  }
  return RR_OK;
}

rr_status Solve::queue_chunk() {
  Work& w = *ws;
  const int F = h->X.F;
  if (op.krylov == RR_KRYLOV_FCG) {
    // flexible CG (the paper's flexible-CG algorithm): direction i is z_i
    // orthogonalized against the m_i previous ones, m_i = max(1, i mod (m+1))
    const int m = fcg_m;
    for (int c = 0; c < chunk; ++c, ++queued) {
      const int i = queued - fcg_base;
      const int slot = i % m;
      double* pi = w.fcg_p + (size_t)slot * F;
      double* qi = w.fcg_ap + (size_t)slot * F;
      FcgWindow win{};
      if (queued > 0 && two_level) {
        int nrz = 0;
        double* sp = nullptr;   // coarse residual snapshots (pair collection)
        if (snap && queued % snap_every == 0 && snap_queued < snap_max)
          sp = snap + (size_t)(snap_queued++) * h->FC;
        // after a fallback no update has run since the last check: its
        // partials may be another solve's
        RR_TRY(precond(100000000 + queued - 1, skip_check ? nullptr : &stage, &nrz, sp));
        skip_check = false;
      }
      if (i > 0) {
        const int mi = std::max(1, i % (m + 1));
        for (int kk = i - mi; kk < i; ++kk) {
          win.p[win.n] = w.fcg_p + (size_t)(kk % m) * F;
          win.ap[win.n] = w.fcg_ap + (size_t)(kk % m) * F;
          win.slot[win.n] = kk % m;
          ++win.n;
        }
        launch_fcg_dots(F, w.z, win, w.parts.dots, w.sc, two_level ? nullptr : &stage, s);
      }
      launch_fcg_dir(F, w.z, w.r, pi, win, w.parts.dots, w.fcg_paps, w.parts.rz, w.sc, s);
      RR_TRY(op_csr(h, w, pf, queued, pi, s));
      Epi e = base_epi(w, lam);
      e.p = pi;
      e.out = qi;
      e.partials = w.parts.pq;
      int npq = 0;
      RR_TRY(op_csc(h, w, pf, queued, EPI_APPLY_DOT, e, s, &npq));
      launch_fcg_update(F, w.x, w.r, pi, qi, w.z, w.e1, w.D, xref, omega, kind, w.sc,
                        w.parts.pq, npq, w.parts.rz, w.fcg_paps, slot, w.parts.upd, s);
    }
    return RR_OK;
  }
  // (a chunk that begins without a pending folded update, a continued
  // solve's first, runs eagerly: the captured chunk begins with one)
  if (op.graph && !pf.on && !snap && (pu_pending || !pu_fold)) {
    // the chunk's launches are the same for every chunk of this solve (all
    // changing state lives in device memory): capture them once per
    // signature, then replay
    GraphKey key{kind, lam, omega, sl ? sl->Ainv : nullptr, xref, op.residual_history, chunk,
                 (sl && w.block) ? sl->Dinv : nullptr, cycle32, pu_fold ? pu_n : -1};
    // the legacy default stream cannot be captured: use the set's own
    // stream, ordered after and before the caller's with events
    hipStream_t gs = s;
    if (!s) {
      if (!w.stream) RR_HIP(hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking));
      if (!w.graph.ev) RR_HIP(hipEventCreateWithFlags(&w.graph.ev, hipEventDisableTiming));
      gs = w.stream;
    }
    if (!w.graph.exec || !(w.graph.key == key)) {
      w.graph.reset();
      const hipStream_t saved = s;
      s = gs;
      RR_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      rr_status cs = queue_chunk_eager(w, F);
      s = saved;
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(gs, &g);
      if (cs != RR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return cs;
      }
      RR_HIP(e);
      w.graph.graph = g;
      RR_HIP(hipGraphInstantiate(&w.graph.exec, g, nullptr, nullptr, 0));
      w.graph.key = key;
      queued -= chunk;   // the captured launches did not run
    }
    if (gs != s) {
      RR_HIP(hipEventRecord(w.graph.ev, s));
      RR_HIP(hipStreamWaitEvent(gs, w.graph.ev, 0));
    }
    RR_HIP(hipGraphLaunch(w.graph.exec, gs));
    if (gs != s) {
      RR_HIP(hipEventRecord(w.graph.ev, gs));
      RR_HIP(hipStreamWaitEvent(s, w.graph.ev, 0));
    }
    queued += chunk;
    return RR_OK;
  }
  return queue_chunk_eager(w, F);
}

rr_status Solve::queue_chunk_eager(Work& w, int F) {
  for (int c = 0; c < chunk; ++c, ++queued) {
    Epi e = base_epi(w, lam);
    e.p = w.p;
    e.out = w.q;
    e.partials = w.parts.pq;
    int npq = 0;
    if (pu_pending) {   // X p = X z + beta X p, then p = z + beta p in the reduction
      const PUpd pu{w.parts.rz, pu_n, w.sc};
      RR_TRY(op_csr(h, w, pf, queued, w.z, s, nullptr, &pu));
      e.r = w.z;
      e.pnew = w.p;
      RR_TRY(op_csc(h, w, pf, queued, EPI_APPLY_DOT_P, e, s, &npq, w.up));
      pu_pending = false;
    } else if (pu_fold) {   // p ready (a continued solve): X p kept for the next direction
      RR_TRY(op_csr(h, w, pf, queued, w.p, s, nullptr, nullptr, w.up));
      RR_TRY(op_csc(h, w, pf, queued, EPI_APPLY_DOT, e, s, &npq, w.up));
    } else {
      RR_TRY(op_csr(h, w, pf, queued, w.p, s));
      RR_TRY(op_csc(h, w, pf, queued, EPI_APPLY_DOT, e, s, &npq));
    }
    launch_pcg_update(F, w.x, w.r, w.p, w.q, w.z, w.e1, w.D, xref, omega, kind, w.sc,
                      w.parts.pq, npq, w.parts.upd, s);
    if (two_level) {
      int nrz = 0;
      double* sp = nullptr;
      if (snap && (queued + 1) % snap_every == 0 && snap_queued < snap_max)
        sp = snap + (size_t)(snap_queued++) * h->FC;
      RR_TRY(precond_two_level(h, w, pf, 100000000 + queued, kind, lam, omega, *sl, w.r, w.z,
                               &stage, &nrz, s, sp));
      if (pu_fold) {
        pu_pending = true;
        pu_n = nrz;
      } else {
        launch_pupdate(F, w.p, w.z, w.sc, w.parts.rz, nrz, 0, nullptr, s);
      }
    } else {
      launch_pupdate(F, w.p, w.z, w.sc, nullptr, 0, 0, &stage, s);
    }
  }
  return RR_OK;
}

rr_status Solve::poll() {
  Scalars& hs = *ws->sc_host;
  RR_HIP(hipMemcpyAsync(&hs, ws->sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  if (hs.done && hs.status == kStatusFallback && kind == PK_LEARNED) {
    // the network's correction made a step fail: the rest of the solve uses
    // the algebraic cycle from the last good iterate, with a fresh
    // flexible-CG history
    fallback_iter = hs.iter;
    kind = PK_VCYCLE;
    stage.kind = kind;
    fcg_base = queued;
    skip_check = true;
    hs.done = 0;
    hs.status = RR_ERR_NOT_CONVERGED;
    RR_HIP(hipMemcpyAsync(ws->sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, s));
    k_smooth<<<cdiv(h->X.F, kBlock), kBlock, 0, s>>>(h->X.F, ws->r, ws->D, omega, ws->e1);
    last_rr = -1.0;
    return RR_OK;
  }
  if (hs.done) {
    done = true;
    return RR_OK;
  }
  if (kind == PK_LEARNED && hs.iter > 0) {
    // a chunk that reduced ||r|| by less than 10 % counts as a stall: the
    // rest of the solve uses the algebraic V(1,1) cycle (flexible CG takes a
    // changing preconditioner), whose first smoother step is formed here
    if (last_rr >= 0.0 && !(hs.rr < 0.81 * last_rr)) {
      fallback_iter = hs.iter;
      kind = PK_VCYCLE;
      stage.kind = kind;
      k_smooth<<<cdiv(h->X.F, kBlock), kBlock, 0, s>>>(h->X.F, ws->r, ws->D, omega, ws->e1);
    }
    last_rr = hs.rr;
  }
  if (queued > hs.limit + 2 * chunk)
    return fail(RR_ERR_DEVICE, "internal: iteration limit passed without the device finishing");
  return RR_OK;
}

rr_status Solve::finish(rr_solve_info* info) {
  Work& w = *ws;
  const int F = h->X.F;
  Scalars& hs = *w.sc_host;
  // exit: w = x and the true residual ||b - A x||
  launch_gather(wout, w.x, h->finv, F, s);
  {
    launch_csr(w.X, w.x, w.u, nullptr, s);
    Epi e = base_epi(w, lam);
    e.p = w.x;
    e.r = w.b;
    e.out = nullptr;
    e.partials = w.parts.tr;
    const int ntr = launch_csc(w.X, w.u, EPI_TRUE, e, nullptr, s);
    launch_finish_true(w.sc, w.parts.tr, ntr, s);
  }
  RR_HIP(hipMemcpyAsync(&hs, w.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  rr_solve_info inf{};
  inf.status = hs.status;
  inf.iters = hs.iter;
  // the V-cycle's two applications after the last update are skipped; the
  // ones before the first iteration are not
  inf.op_applies = (kind == PK_VCYCLE || kind == PK_LEARNED) ? 3 * hs.iter
                   : kind == PK_ROUGHER ? (1 + w.rsteps) * hs.iter : hs.iter;
  inf.relres = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
  inf.true_relres = hs.bb > 0 ? std::sqrt(hs.true_rr / hs.bb) : 0.0;
  inf.err = hs.ref2 > 0 ? std::sqrt(hs.ee / hs.ref2) : 0.0;
  inf.omega = omega;
  inf.coarse_ms = coarse_ms;
  inf.fallback_iter = fallback_iter;
  if (pf.on) {
    // count only launches that ran: iteration tags below the final count
    auto acc = [&](const std::vector<std::pair<int, int>>& v, double* avg, double* gavg, int* n) {
      double tot = 0.0, gtot = 0.0;
      int cnt = 0;
      for (auto& pr : v) {
        const int tag = pr.second;
        const bool ran = (tag < 0) || (tag < 100000000 ? tag < hs.iter : tag - 100000000 + 1 < hs.iter);
        if (!ran) continue;
        float ms = 0.f, gms = 0.f;
        const hipEvent_t* ev = &h->ev_pool[3 * pr.first];
        if (hipEventElapsedTime(&ms, ev[0], ev[2]) == hipSuccess &&
            hipEventElapsedTime(&gms, ev[0], ev[1]) == hipSuccess) {
          tot += ms;
          gtot += gms;
          ++cnt;
        }
      }
      *avg = cnt ? tot / cnt : 0.0;
      *gavg = cnt ? gtot / cnt : 0.0;
      *n = cnt;
    };
    acc(pf.csr, &inf.csr_avg_ms, &inf.csr_gather_avg_ms, &inf.csr_launches);
    acc(pf.csc, &inf.csc_avg_ms, &inf.csc_gather_avg_ms, &inf.csc_launches);
    if ((op.profile == 2 || op.profile == 3) && h->X.sliced) {
      // back-to-back launches of each gather kernel on the final x and u = X x
      constexpr int kReps = 20;
      int ti = 0;
      RR_TRY(prof_pair(h, pf, &ti));
      const hipEvent_t* ev = &h->ev_pool[3 * ti];
      float ms = 0.f;
      RR_HIP(hipEventRecord(ev[0], s));
      for (int i = 0; i < kReps; ++i) launch_rows(w.X.rows, w.x, w.u, nullptr, nullptr, s);
      RR_HIP(hipEventRecord(ev[1], s));
      if (op.profile == 3) {   // the column pass with its reduction (q = X^T u + lambda x, <x, q>)
        Epi e = base_epi(w, lam);
        e.p = w.x;
        e.out = w.q;
        e.partials = w.parts.pq;
        for (int i = 0; i < kReps; ++i) (void)launch_sell(w.X.sell_csc, w.u, EPI_APPLY_DOT, e, nullptr, s, nullptr, nullptr);
      } else {
        for (int i = 0; i < kReps; ++i) launch_sell_gather(w.X.sell_csc, w.u, s);
      }
      RR_HIP(hipEventRecord(ev[2], s));
      RR_HIP(hipEventSynchronize(ev[2]));
      RR_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
      inf.csr_gather_avg_ms = ms / kReps;
      RR_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
      inf.csc_gather_avg_ms = ms / kReps;
    }
  }
  inf.ms = now_ms() - t0;
  if (info) *info = inf;
  if (hs.status == RR_ERR_NOT_CONVERGED)
    return fail(RR_ERR_NOT_CONVERGED, "max_iter reached before the tolerance");
  if (hs.status == RR_ERR_BREAKDOWN)
    return fail(RR_ERR_BREAKDOWN, "breakdown: <p,Ap> or <r,z> not positive");
  return RR_OK;
}

}  // namespace

namespace rr {

// ---- coarse Gram matrix of a valued X ---------------------------------------

// v = P e_s: the scaled indicator of cluster s (per-feature weights pw for
// least-squares interpolation)
__global__ void k_cluster_vec(int F, const int* __restrict__ labels, const double* __restrict__ cscale,
                              const double* __restrict__ pw, int cl, double* __restrict__ v) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) v[j] = (labels[j] == cl) ? (pw ? pw[j] : cscale[cl]) : 0.0;
}

// c = P^T v: each cluster's sum scaled by 1/sqrt(n_s), or each member
// weighted by its own p_j (the merge path's per-entry values)
void launch_restrict(const rr_handle* h, const MergePlan& mp, const double* v, double* out,
                     const int* done, hipStream_t s) {
  Epi er{};
  er.out = out;
  if (h->lsw) {
    launch_segsum(mp, h->coff + 1, h->perm, h->lsw_perm, v, EPI_STORE, er, done, s);
  } else {
    er.scale = h->cscale;
    launch_segsum(mp, h->coff + 1, h->perm, nullptr, v, EPI_SCALE, er, done, s);
  }
}

void launch_restrict_sorted(const rr_handle* h, const MergePlan& mp, const double* v, double* out,
                            const int* done, hipStream_t s) {
  Epi er{};
  er.out = out;
  if (h->lsw) {
    launch_segsum(mp, h->coff + 1, nullptr, h->lsw_perm, v, EPI_STORE, er, done, s);
  } else {
    er.scale = h->cscale;
    launch_segsum(mp, h->coff + 1, nullptr, nullptr, v, EPI_SCALE, er, done, s);
  }
}

// K = P^T X^T X P column by column: K e_s = P^T X^T (X (P e_s)) with the
// operator's passes and the restriction (FP64; K is symmetric, so column s is
// stored as row s).
rr_status build_coarse_gram_valued(rr_handle* h, hipStream_t s) {
  const int F = h->X.F, N = h->X.N, fc = h->FC;
  double *v = nullptr, *u = nullptr, *t = nullptr;
  RR_TRY(dalloc(&v, F));
  RR_TRY(dalloc(&u, N));
  RR_TRY(dalloc(&t, F));
  for (int c = 0; c < fc; ++c) {
    k_cluster_vec<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, h->labels, h->cscale, h->lsw, c, v);
    launch_csr(h->X, v, u, nullptr, s);
    Epi e{};
    e.out = t;
    launch_csc(h->X, u, EPI_STORE, e, nullptr, s);
    launch_restrict(h, h->restrict_plan, t, h->K + (size_t)c * fc, nullptr, s);
  }
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  dfree(v);
  dfree(u);
  dfree(t);
  return RR_OK;
}

}  // namespace rr

namespace {

// ---- mixed precision: FP32 inner PCG inside FP64 iterative refinement ------

rr_status ensure_f32(rr_handle* h, Work& w) {
  IrVectors& f = w.f32;
  if (f.x) return RR_OK;
  const int F = h->X.F, N = h->X.N;
  RR_TRY(dalloc(&f.x, F)); RR_TRY(dalloc(&f.r, F)); RR_TRY(dalloc(&f.p, F));
  RR_TRY(dalloc(&f.q, F)); RR_TRY(dalloc(&f.z, F)); RR_TRY(dalloc(&f.e1, F));
  RR_TRY(dalloc(&f.e2, F)); RR_TRY(dalloc(&f.D, F));
  RR_TRY(dalloc(&f.u, N));
  RR_TRY(dalloc(&f.part_cols, h->X.sell_csc.nout));
  return RR_OK;
}

// z32 = B r32 (V(1,1), FP32 vectors, FP64 coarse solve); <r,z> partials in
// parts.rz, their count in *n_rz.
rr_status precond32(rr_handle* h, Work& w, double lam, double omega, const LambdaSlot& sl,
                    const StageArgs* stage, int* n_rz, hipStream_t s) {
  IrVectors& f = w.f32;
  const int F = h->X.F;
  const int* done = &w.sc->done;
  Epi32 e{};
  e.lam = lam;
  e.out = f.u;
  launch_rows32(w.X.rows, f.e1, f.u, done, s, stage);
  Epi32 er{};
  er.lam = lam;
  er.p = f.e1;
  er.r = f.r;
  er.out64 = w.rho;
  launch_sell32(w.X.sell_csc, f.part_cols, f.u, EPI_RESID, er, done, s);
  Epi ec{};
  ec.scale = h->cscale;
  ec.out = w.c;
  launch_segsum(w.rplan, h->coff + 1, h->perm, nullptr, w.rho, EPI_SCALE, ec, done, s);
  launch_gemv(h->FC, sl.Ainv, w.c, w.yc, done, s);
  launch_prolong32(F, h->labels, h->cscale, w.yc, f.e1, f.e2, done, s);
  if (h->crow.nlayer > 0)   // X e2 = X e1 + X P yc, u still holding X e1
    launch_cluster_rows32(h, w.yc, f.u, done, s);
  else
    launch_rows32(w.X.rows, f.e2, f.u, done, s);
  Epi32 ep{};
  ep.lam = lam;
  ep.omega = omega;
  ep.p = f.e2;
  ep.r = f.r;
  ep.D = f.D;
  ep.out = f.z;
  ep.partials = w.parts.rz;
  *n_rz = launch_sell32(w.X.sell_csc, f.part_cols, f.u, EPI_POST, ep, done, s);
  return RR_OK;
}

rr_status solve_ir(rr_handle* h, Work& w, double lam, const double* rhs, double* wout,
                   const rr_solve_opts& op, rr_solve_info* info, hipStream_t s) {
  const double t0 = now_ms();
  RR_TRY(check_lambda(lam, false));
  if (!rhs || !wout) return fail(RR_ERR_INVALID_ARG, "null rhs or w");
  if (!h->X.binary)
    return fail(RR_ERR_UNSUPPORTED, "single-precision inner solves are built for 0/1 X only");
  if (h->X.rw) return fail(RR_ERR_UNSUPPORTED, "single-precision inner solves are built for unweighted X");
  if (h->lsw)
    return fail(RR_ERR_UNSUPPORTED,
                "single-precision inner solves use the adjusted square-root average interpolation");
  const int kind = op.precond;
  if (kind != PK_NONE && kind != PK_JACOBI && kind != PK_VCYCLE)
    return fail(RR_ERR_UNSUPPORTED, "iterative refinement supports the none, Jacobi and V(1,1) preconditioners");
  if (kind == PK_VCYCLE && h->FC == 0)
    return fail(RR_ERR_INVALID_ARG, "two-level preconditioner needs a coarse level (n_clusters > 0)");
  if (op.krylov != RR_KRYLOV_PCG) return fail(RR_ERR_UNSUPPORTED, "iterative refinement runs PCG inner solves");
  if (op.smoother != RR_SMOOTHER_POINT)
    return fail(RR_ERR_UNSUPPORTED, "iterative refinement smooths with the point smoother");
  if (op.x_ref || op.residual_history || op.fixed_iters)
    return fail(RR_ERR_INVALID_ARG, "x_ref, residual_history and fixed_iters are not used with refinement");
  if (op.max_iter < 0 || op.chunk < 0 || op.tol < 0 || op.inner_tol < 0 || op.inner_tol >= 1)
    return fail(RR_ERR_INVALID_ARG, "bad refinement option");
  const double tol = op.tol > 0 ? op.tol : 1e-10;
  const double inner_tol = op.inner_tol > 0 ? op.inner_tol : 1e-4;
  const int max_inner = op.max_iter > 0 ? op.max_iter : 10000;
  const int chunk = op.chunk > 0 ? op.chunk : 8;
  constexpr int kMaxSteps = 40;
  const int F = h->X.F;
  LambdaSlot* sl = nullptr;
  double coarse_ms = 0.0, omega = op.omega;
  if (kind == PK_VCYCLE) {
    RR_TRY(get_slot(h, w.X, lam, &sl, &coarse_ms, s));
    if (omega == 0.0) omega = sl->omega;
  }
  if (!std::isfinite(omega) || omega < 0.0) return fail(RR_ERR_INVALID_ARG, "omega must be finite and >= 0");
  RR_TRY(ensure_f32(h, w));
  if (sl) sl->in_use++;
  struct Unpin {
    LambdaSlot* sl;
    ~Unpin() { if (sl) sl->in_use--; }
  } unpin{sl};
  if (op.rhs_is_b) {
    launch_gather(w.b, rhs, h->fperm, F, s);
  } else {
    Epi e{};
    e.out = w.b;
    launch_csc(w.X, rhs, EPI_STORE, e, nullptr, s);
  }
  // outer state: x = 0, r = b, ||b||^2 (FP64)
  Scalars& hs = *w.sc_host;
  std::memset(&hs, 0, sizeof(Scalars));
  RR_HIP(hipMemcpyAsync(w.sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, s));
  const int nv = w.parts.n_vec;
  launch_colnorm_diag(F, h->colnorm, lam, w.D, s);
  launch_pcg_init(F, w.b, w.x, w.r, w.p, w.z, w.e1, w.D, nullptr, 0.0, PK_NONE, w.parts.init, s);
  launch_finish_init(w.sc, w.parts.init, nv, nullptr, PK_NONE, s);
  RR_HIP(hipMemcpyAsync(&hs, w.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  const double bb = hs.bb;
  int status = RR_ERR_NOT_CONVERGED, steps = 0, inner_total = 0;
  double rr_true = bb;
  if (!(bb > 0.0)) {
    status = (bb == 0.0) ? RR_OK : RR_ERR_BREAKDOWN;
    rr_true = 0.0;
  }
  IrVectors& f = w.f32;
  StageArgs stage{w.sc, w.parts.upd, nv, nullptr, kind};
  while (status == RR_ERR_NOT_CONVERGED && steps < kMaxSteps) {
    // inner solve A d = r with FP32 vectors, to relative residual inner_tol
    std::memset(&hs, 0, sizeof(Scalars));
    hs.tol2 = inner_tol * inner_tol;
    hs.limit = max_inner;
    hs.status = RR_ERR_NOT_CONVERGED;
    RR_HIP(hipMemcpyAsync(w.sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, s));
    launch_ir_init(F, w.r, h->colnorm, lam, omega, kind, f, w.parts.init, s);
    launch_finish_init(w.sc, w.parts.init, nv, nullptr, kind, s);
    if (kind == PK_VCYCLE) {
      int nrz = 0;
      RR_TRY(precond32(h, w, lam, omega, *sl, nullptr, &nrz, s));
      launch_ir_pupdate(F, f.p, f.z, w.sc, w.parts.rz, nrz, 1, nullptr, s);
    } else {
      launch_ir_pupdate(F, f.p, f.z, w.sc, w.parts.init + 2 * nv, nv, 1, nullptr, s);
    }
    int queued = 0;
    for (;;) {
      for (int c = 0; c < chunk; ++c, ++queued) {
        const int* done = &w.sc->done;
        Epi32 e{};
        e.out = f.u;
        launch_rows32(w.X.rows, f.p, f.u, done, s);
        Epi32 eq{};
        eq.lam = lam;
        eq.p = f.p;
        eq.out = f.q;
        eq.partials = w.parts.pq;
        const int npq = launch_sell32(w.X.sell_csc, f.part_cols, f.u, EPI_APPLY_DOT, eq, done, s);
        launch_ir_update(F, f, omega, kind, w.sc, w.parts.pq, npq, w.parts.upd, s);
        if (kind == PK_VCYCLE) {
          int nrz = 0;
          RR_TRY(precond32(h, w, lam, omega, *sl, &stage, &nrz, s));
          launch_ir_pupdate(F, f.p, f.z, w.sc, w.parts.rz, nrz, 0, nullptr, s);
        } else {
          launch_ir_pupdate(F, f.p, f.z, w.sc, nullptr, 0, 0, &stage, s);
        }
      }
      RR_HIP(hipMemcpyAsync(&hs, w.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
      RR_HIP(hipStreamSynchronize(s));
      RR_HIP(hipGetLastError());
      if (hs.done) break;
      if (queued > hs.limit + 2 * chunk)
        return fail(RR_ERR_DEVICE, "internal: iteration limit passed without the device finishing");
    }
    inner_total += hs.iter;
    ++steps;
    if (hs.status == RR_ERR_BREAKDOWN && hs.iter == 0) {
      status = RR_ERR_BREAKDOWN;
      break;
    }
    // x += d; r = b - A x in FP64, ||r||^2
    launch_ir_accumulate(F, w.x, f.x, s);
    launch_csr(w.X, w.x, w.u, nullptr, s);
    Epi e = base_epi(w, lam);
    e.p = w.x;
    e.r = w.b;
    e.out = w.r;
    e.partials = w.parts.tr;
    const int ntr = launch_csc(w.X, w.u, EPI_TRUE, e, nullptr, s);
    launch_finish_true(w.sc, w.parts.tr, ntr, s);
    RR_HIP(hipMemcpyAsync(&hs, w.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
    RR_HIP(hipGetLastError());
    rr_true = hs.true_rr;
    if (!(rr_true == rr_true)) {
      status = RR_ERR_BREAKDOWN;
      break;
    }
    if (rr_true <= tol * tol * bb) status = RR_OK;
  }
  launch_gather(wout, w.x, h->finv, F, s);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  rr_solve_info inf{};
  inf.status = status;
  inf.iters = inner_total;
  inf.ir_steps = steps;
  inf.op_applies = (kind == PK_VCYCLE ? 3 * inner_total : inner_total) + steps;
  inf.relres = bb > 0 ? std::sqrt(rr_true / bb) : 0.0;
  inf.true_relres = inf.relres;
  inf.omega = omega;
  inf.coarse_ms = coarse_ms;
  inf.ms = now_ms() - t0;
  if (info) *info = inf;
  if (status == RR_ERR_NOT_CONVERGED)
    return fail(RR_ERR_NOT_CONVERGED, "refinement steps exhausted before the tolerance");
  if (status == RR_ERR_BREAKDOWN) return fail(RR_ERR_BREAKDOWN, "breakdown in refinement");
  return RR_OK;
}

rr_status solve_impl(rr_handle* h, double lam, const double* rhs, double* wout,
                     const rr_solve_opts* o, rr_solve_info* info, hipStream_t s) {
  if (o && o->precision == RR_PREC_F32_IR) return solve_ir(h, h->w, lam, rhs, wout, *o, info, s);
  if (o && o->precision != RR_PREC_F64 && o->precision != RR_PREC_F32_CYCLE)
    return fail(RR_ERR_INVALID_ARG, "unknown precision");
  Solve sv;
  sv.h = h;
  sv.ws = &h->w;
  sv.lam = lam;
  sv.rhs = rhs;
  sv.wout = wout;
  if (o) sv.op = *o;
  sv.s = s;
  rr_status st = sv.begin();
  while (st == RR_OK && !sv.done) {
    st = sv.queue_chunk();
    if (st == RR_OK) st = sv.poll();
  }
  if (st == RR_OK) st = sv.finish(info);
  sv.release();
  return st;
}

// Problems run concurrently, each in its own work set (the k-th problem on
// a handle in the k-th set) on that set's stream, with their iteration
// chunks queued round-robin.  More than kMaxSets problems on one handle run
// in later waves.
constexpr int kMaxSets = 8;

rr_status solve_batched_persistent(int nprob, rr_handle* const* hs, const double* lams,
                                   const double* const* rhs, double* const* ws, const rr_solve_opts& op,
                                   rr_solve_info* infos, hipStream_t caller, bool noalloc = false);

rr_status solve_batched_impl(int nprob, rr_handle* const* hs, const double* lams,
                             const double* const* rhs, double* const* ws, const rr_solve_opts* o,
                             rr_solve_info* infos, hipStream_t caller) {
  if (nprob < 0) return fail(RR_ERR_INVALID_ARG, "nprob must be >= 0");
  if (nprob == 0) return RR_OK;
  if (!hs || !lams || !rhs || !ws) return fail(RR_ERR_INVALID_ARG, "null batch array");
  rr_solve_opts op{};
  if (o) op = *o;
  if (op.x_ref || op.residual_history)
    return fail(RR_ERR_INVALID_ARG, "x_ref and residual_history are per-problem buffers: use rr_solve");
  if (op.precision != RR_PREC_F64)
    return fail(RR_ERR_UNSUPPORTED, "batched solves run in FP64");
  op.profile = 0;
  for (int i = 0; i < nprob; ++i) {
    if (!hs[i]) return fail(RR_ERR_INVALID_ARG, "null handle in batch");
    RR_TRY(check_sparse(hs[i]));
  }
  if (op.persistent < 0 || op.persistent > 2) return fail(RR_ERR_INVALID_ARG, "persistent must be 0, 1 or 2");
  if (op.persistent) return solve_batched_persistent(nprob, hs, lams, rhs, ws, op, infos, caller);
  std::vector<int> wave(nprob, 0), set(nprob, 0);
  int nwaves = 0;
  for (int i = 0; i < nprob; ++i) {
    int k = 0;
    for (int j = 0; j < i; ++j) k += (hs[j] == hs[i]);
    wave[i] = k / kMaxSets;
    set[i] = k % kMaxSets;
    nwaves = std::max(nwaves, wave[i] + 1);
  }
  hipEvent_t ev;
  RR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  RR_HIP(hipEventRecord(ev, caller));
  rr_status first_bad = RR_OK;
  for (int wv = 0; wv < nwaves; ++wv) {
    std::vector<std::unique_ptr<Solve>> sv;
    std::vector<int> idx;
    for (int i = 0; i < nprob; ++i) {
      if (wave[i] != wv) continue;
      rr_handle* h = hs[i];
      Work* w = nullptr;
      {
        MemScope ms(&h->mem);
        RR_TRY(get_work_set(h, set[i], &w));
      }
      hipStream_t* st = (set[i] == 0) ? &h->bstream : &w->stream;
      if (!*st) RR_HIP(hipStreamCreateWithFlags(st, hipStreamNonBlocking));
      RR_HIP(hipStreamWaitEvent(*st, ev, 0));
      std::unique_ptr<Solve> x(new Solve());
      x->h = h;
      x->ws = w;
      x->lam = lams[i];
      x->rhs = rhs[i];
      x->wout = ws[i];
      x->op = op;
      x->s = *st;
      sv.push_back(std::move(x));
      idx.push_back(i);
    }
    std::vector<rr_status> st(sv.size(), RR_OK);
    for (size_t j = 0; j < sv.size(); ++j) {
      MemScope ms(&sv[j]->h->mem);
      st[j] = sv[j]->begin();
    }
    for (;;) {
      bool active = false;
      for (size_t j = 0; j < sv.size(); ++j)
        if (st[j] == RR_OK && !sv[j]->done) {
          st[j] = sv[j]->queue_chunk();
          active = true;
        }
      if (!active) break;
      for (size_t j = 0; j < sv.size(); ++j)
        if (st[j] == RR_OK && !sv[j]->done) st[j] = sv[j]->poll();
    }
    for (size_t j = 0; j < sv.size(); ++j) {
      rr_solve_info inf{};
      if (st[j] == RR_OK) {
        st[j] = sv[j]->finish(&inf);
      } else {
        (void)hipStreamSynchronize(sv[j]->s);
        inf.status = st[j];
      }
      sv[j]->release();
      if (infos) infos[idx[j]] = inf;
      if (st[j] != RR_OK && first_bad == RR_OK) first_bad = st[j];
    }
    // the next wave and the caller's later work wait for this wave
    for (size_t j = 0; j < sv.size(); ++j) {
      RR_HIP(hipEventRecord(ev, sv[j]->s));
      RR_HIP(hipStreamWaitEvent(caller, ev, 0));
    }
    RR_HIP(hipEventRecord(ev, caller));
  }
  RR_HIP(hipEventDestroy(ev));
  return first_bad;
}

// ---- persistent batched solve ------------------------------------------------

// Device buffers of the persistent batched solve, kept by the library per
// device and grown when a larger batch arrives (the solve itself allocates
// nothing once they are large enough).
struct BatchBuffers {
  BatchProb* probs = nullptr;
  int* order = nullptr;
  BatchOut* out = nullptr;
  int* queue = nullptr;
  int cap = 0;
  hipStream_t stream = nullptr;   // capture stream of the launch graph
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_n = -1, graph_grid = -1;
  MemCtx mem;   // where the buffers came from
};
std::mutex g_batch_mu;
BatchBuffers g_batch[64];

rr_status batch_buffers(int dev, int n, BatchBuffers** out) {
  if (dev < 0 || dev >= 64) return fail(RR_ERR_UNSUPPORTED, "device index above 63");
  BatchBuffers& b = g_batch[dev];
  if (b.cap < n) {
    MemScope old_mem(&b.mem);
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.graph_n = b.graph_grid = -1;
    dfree(b.probs);
    dfree(b.order);
    dfree(b.out);
    b.probs = nullptr;
    b.order = nullptr;
    b.out = nullptr;
    b.cap = 0;
    if (b.queue) (void)dev_free(b.queue);
    b.queue = nullptr;
    b.mem = default_mem();
    MemScope new_mem(&b.mem);
    const int cap = std::max(n, 64);
    RR_HIP(dmalloc(&b.probs, sizeof(BatchProb) * cap));
    RR_HIP(dmalloc(&b.order, sizeof(int) * cap));
    RR_HIP(dmalloc(&b.out, sizeof(BatchOut) * cap));
    RR_HIP(dmalloc(&b.queue, sizeof(int)));
    b.cap = cap;
  }
  if (!b.stream) RR_HIP(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
  if (!b.ev) RR_HIP(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
  *out = &b;
  return RR_OK;
}

// All problems in one persistent kernel launch (captured once per batch size
// into a HIP graph and replayed): one workgroup per problem at a time, the
// problems taken longest first.
rr_status solve_batched_persistent(int nprob, rr_handle* const* hs, const double* lams,
                                   const double* const* rhs, double* const* ws, const rr_solve_opts& op,
                                   rr_solve_info* infos, hipStream_t caller, bool noalloc) {
  const double t0 = now_ms();
  if (noalloc) {
    // nothing may be allocated: every work set and coarse factor must exist
    if (nprob > kStaticProblems)
      return fail(RR_ERR_INVALID_ARG, "the allocation-free batched solve takes at most 2048 problems");
    for (int i = 0; i < nprob; ++i) {
      int k = 0, nl = 0;
      for (int j = 0; j < i; ++j) k += (hs[j] == hs[i]);
      if (k > (int)hs[i]->extra_sets.size())
        return fail(RR_ERR_WORKSPACE, "a handle appears more often than its reserved work sets allow "
                                      "(rr_setup_opts.reserve_sets)");
      for (int j = 0; j < nprob; ++j) {
        if (hs[j] != hs[i]) continue;
        bool seen = false;
        for (int q = 0; q < j; ++q) seen = seen || (hs[q] == hs[i] && lams[q] == lams[j]);
        nl += !seen;
      }
      if (op.precond == RR_PRECOND_VCYCLE && nl > (int)hs[i]->slots.size())
        return fail(RR_ERR_WORKSPACE, "more distinct lambdas on a handle than its lambda_slots");
    }
  }
  if (op.krylov != RR_KRYLOV_PCG || op.precision != RR_PREC_F64 || op.smoother != RR_SMOOTHER_POINT)
    return fail(RR_ERR_UNSUPPORTED, "the persistent batched solve runs FP64 PCG with the point smoother");
  if (op.precond != RR_PRECOND_VCYCLE && op.precond != RR_PRECOND_JACOBI)
    return fail(RR_ERR_UNSUPPORTED, "the persistent batched solve runs the V(1,1) or Jacobi preconditioner");
  if (op.fixed_iters < 0 || op.max_iter < 0 || op.tol < 0 || op.hybrid_iters < 0)
    return fail(RR_ERR_INVALID_ARG, "negative option");
  const double tol = op.tol > 0 ? op.tol : 1e-10;
  const int max_iter = op.fixed_iters > 0 ? op.fixed_iters : (op.max_iter > 0 ? op.max_iter : 10000);
  int dev = 0;
  RR_HIP(hipGetDevice(&dev));
  std::vector<BatchProb> pv(nprob);
  std::vector<long long> cost(nprob);
  std::vector<LambdaSlot*> used;
  rr_status res = RR_OK;
  for (int i = 0; i < nprob && res == RR_OK; ++i) {
    rr_handle* h = hs[i];
    const Sparse& X = h->X;
    if (!X.binary || !X.bplan.csplit) {
      res = fail(RR_ERR_UNSUPPORTED, "the persistent batched solve needs 0/1 X with at most 8192 features");
      break;
    }
    if (h->device != dev) {
      res = fail(RR_ERR_INVALID_ARG, "every handle of a persistent batch must live on the current device");
      break;
    }
    if (X.rw || h->lsw) {
      res = fail(RR_ERR_UNSUPPORTED, "the persistent batched solve runs unweighted X with P of the square-root average");
      break;
    }
    const bool vc = op.precond == RR_PRECOND_VCYCLE;
    if (vc && (h->FC == 0 || 2 * h->FC > kBatchRows)) {
      res = fail(RR_ERR_INVALID_ARG, "V(1,1) in the persistent batched solve needs 1 <= n_coarse <= 5120");
      break;
    }
    res = check_lambda(lams[i], false);
    if (res != RR_OK) break;
    if (!rhs[i] || !ws[i]) {
      res = fail(RR_ERR_INVALID_ARG, "null rhs or w");
      break;
    }
    int k = 0;
    for (int j = 0; j < i; ++j) k += (hs[j] == h);
    MemScope ms(&h->mem);
    Work* w = nullptr;
    res = get_work_set(h, k, &w);
    if (res != RR_OK) break;
    BatchProb& P = pv[i];
    std::memset(&P, 0, sizeof(P));
    P.N = X.N;
    P.F = X.F;
    P.FC = vc ? h->FC : 0;
    P.nchunk = X.bplan.nchunk;
    P.grow = X.bplan.grow;
    for (int c = 0; c < 3; ++c) P.cls[c] = X.bplan.cls[c];
    P.kind = vc ? 1 : 0;
    P.rhs_is_b = op.rhs_is_b ? 1 : 0;
    P.max_iter = max_iter;
    P.fixed = op.fixed_iters > 0 ? 1 : 0;
    P.rp = X.row_ptr;
    P.ci = X.bplan.ci16;
    P.ri = X.bplan.ri16;
    P.csplit = X.bplan.csplit;
    P.perm = h->perm;
    P.coff = h->coff;
    P.labels = h->labels;
    P.fperm = h->fperm;
    P.finv = h->finv;
    P.cscale = h->cscale;
    P.colnorm = h->colnorm;
    P.rhs = rhs[i];
    P.lam = lams[i];
    P.tol2 = op.fixed_iters > 0 ? 0.0 : tol * tol;
    P.omega = op.omega;
    if (vc) {
      LambdaSlot* sl = nullptr;
      double ms = 0.0;
      res = get_slot(h, h->X, lams[i], &sl, &ms, caller);
      if (res != RR_OK) break;
      sl->in_use++;
      used.push_back(sl);
      P.Ainv = sl->Ainv;
      if (P.omega == 0.0) P.omega = sl->omega;
    }
    if (!std::isfinite(P.omega) || P.omega < 0.0) {
      res = fail(RR_ERR_INVALID_ARG, "omega must be finite and >= 0");
      break;
    }
    P.w = ws[i];
    P.x = w->x;
    P.r = w->r;
    P.p = w->p;
    P.z = w->z;
    P.e1 = w->e1;
    P.b = w->b;
    P.t = w->q;
    cost[i] = (long long)X.nnz + X.N + X.F;
  }
  BatchBuffers* bb = nullptr;
  BatchScratch scratch;
  std::unique_lock<std::mutex> lk(g_batch_mu);
  if (res == RR_OK) res = noalloc ? batch_scratch(&scratch) : batch_buffers(dev, nprob, &bb);
  if (res == RR_OK && noalloc) {
    // the static scratch stands in for the library's buffers; no graph
    static BatchBuffers view;
    view = BatchBuffers{};
    view.probs = scratch.probs;
    view.order = scratch.order;
    view.out = scratch.out;
    view.queue = scratch.queue;
    view.cap = scratch.cap;
    bb = &view;
  }
  if (res == RR_OK) {
    std::vector<int> order(nprob);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = std::max(1, std::min(nprob, ncu));
    if (op.persistent == 2 && !noalloc) {
      // hybrid: a problem leaves the kernel after cap_i = B / cost_i
      // iterations, B = hybrid_iters x (total cost / workgroups): the kernel
      // then ends near the balanced time of hybrid_iters iterations per
      // problem, and the few problems that need many more continue with
      // the stream kernels, which spread one problem over the whole GPU.
      // The caps depend on the sizes only, so results are reproducible.
      constexpr int kMinCap = 16;
      const double iters = op.hybrid_iters > 0 ? op.hybrid_iters : 512.0;
      double tot = 0.0;
      for (int i = 0; i < nprob; ++i) tot += (double)cost[i];
      const double B = iters * tot / grid;
      for (int i = 0; i < nprob; ++i) {
        const double c = std::ceil(B / std::max<double>(1.0, (double)cost[i]));
        pv[i].cap = c >= (double)pv[i].max_iter ? 0 : std::max(kMinCap, (int)c);
      }
    }
    auto run = [&]() -> rr_status {
      RR_HIP(hipMemcpyAsync(bb->probs, pv.data(), sizeof(BatchProb) * nprob, hipMemcpyHostToDevice, caller));
      RR_HIP(hipMemcpyAsync(bb->order, order.data(), sizeof(int) * nprob, hipMemcpyHostToDevice, caller));
      if (op.graph && !noalloc) {
        if (!bb->exec || bb->graph_n != nprob || bb->graph_grid != grid) {
          if (bb->exec) (void)hipGraphExecDestroy(bb->exec);
          if (bb->graph) (void)hipGraphDestroy(bb->graph);
          bb->exec = nullptr;
          bb->graph = nullptr;
          RR_HIP(hipStreamBeginCapture(bb->stream, hipStreamCaptureModeThreadLocal));
          launch_batch_solve(bb->probs, bb->order, nprob, bb->queue, bb->out, grid, bb->stream);
          hipGraph_t g = nullptr;
          RR_HIP(hipStreamEndCapture(bb->stream, &g));
          bb->graph = g;
          RR_HIP(hipGraphInstantiate(&bb->exec, g, nullptr, nullptr, 0));
          bb->graph_n = nprob;
          bb->graph_grid = grid;
        }
        RR_HIP(hipEventRecord(bb->ev, caller));
        RR_HIP(hipStreamWaitEvent(bb->stream, bb->ev, 0));
        RR_HIP(hipGraphLaunch(bb->exec, bb->stream));
        RR_HIP(hipEventRecord(bb->ev, bb->stream));
        RR_HIP(hipStreamWaitEvent(caller, bb->ev, 0));
      } else {
        launch_batch_solve(bb->probs, bb->order, nprob, bb->queue, bb->out, grid, caller);
      }
      RR_HIP(hipGetLastError());
      return RR_OK;
    };
    res = run();
    if (res == RR_OK) {
      std::vector<BatchOut> out(nprob);
      RR_HIP(hipMemcpyAsync(out.data(), bb->out, sizeof(BatchOut) * nprob, hipMemcpyDeviceToHost, caller));
      RR_HIP(hipStreamSynchronize(caller));
      int clock_khz = 0;
      (void)hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
      // problems that left the kernel at their cap: the PCG recurrence goes
      // on from the work set's x, r, p and the recorded <r,z>, with the
      // stream kernels (every problem on its work set's stream)
      std::vector<rr_solve_info> cont(nprob);
      std::vector<char> continued(nprob, 0);
      {
        std::vector<std::unique_ptr<Solve>> sv;
        std::vector<std::unique_ptr<Solve::Resume>> rs;
        std::vector<int> idx;
        for (int i = 0; i < nprob && res == RR_OK; ++i) {
          if (out[i].status != kStatusYield) continue;
          rr_handle* h = hs[i];
          int k = 0;
          for (int j = 0; j < i; ++j) k += (hs[j] == h);
          Work* w = nullptr;
          {
            MemScope ms(&h->mem);
            res = get_work_set(h, k, &w);
          }
          if (res != RR_OK) break;
          hipStream_t* st = (k == 0) ? &h->bstream : &w->stream;
          if (!*st) RR_HIP(hipStreamCreateWithFlags(st, hipStreamNonBlocking));
          std::unique_ptr<Solve::Resume> r(new Solve::Resume{out[i].iters, out[i].rz, out[i].bb,
                                                             out[i].relres * out[i].relres * out[i].bb});
          std::unique_ptr<Solve> x(new Solve());
          x->h = h;
          x->ws = w;
          x->lam = lams[i];
          x->rhs = rhs[i];
          x->wout = ws[i];
          x->op = op;
          x->op.omega = pv[i].omega;
          x->s = *st;
          x->resume = r.get();
          rs.push_back(std::move(r));
          sv.push_back(std::move(x));
          idx.push_back(i);
        }
        std::vector<rr_status> st(sv.size(), RR_OK);
        for (size_t j = 0; j < sv.size(); ++j) {
          MemScope ms(&sv[j]->h->mem);
          st[j] = sv[j]->begin();
        }
        for (;;) {
          bool active = false;
          for (size_t j = 0; j < sv.size(); ++j)
            if (st[j] == RR_OK && !sv[j]->done) {
              MemScope ms(&sv[j]->h->mem);
              st[j] = sv[j]->queue_chunk();
              active = true;
            }
          if (!active) break;
          for (size_t j = 0; j < sv.size(); ++j)
            if (st[j] == RR_OK && !sv[j]->done) st[j] = sv[j]->poll();
        }
        for (size_t j = 0; j < sv.size(); ++j) {
          rr_solve_info inf{};
          if (st[j] == RR_OK) {
            MemScope ms(&sv[j]->h->mem);
            (void)sv[j]->finish(&inf);   // its status is in inf
          } else {
            (void)hipStreamSynchronize(sv[j]->s);
            inf.status = st[j];
          }
          sv[j]->release();
          cont[idx[j]] = inf;
          continued[idx[j]] = 1;
        }
      }
      for (int i = 0; i < nprob; ++i) {
        int st = continued[i] ? cont[i].status : out[i].status;
        if (!continued[i] && op.fixed_iters > 0 && st == RR_ERR_NOT_CONVERGED && out[i].iters == op.fixed_iters)
          st = RR_OK;
        const double kernel_ms =
            clock_khz > 0 ? (double)(out[i].t_end - out[i].t_begin) / clock_khz : now_ms() - t0;
        if (infos && continued[i]) {
          rr_solve_info inf = cont[i];
          inf.ms += kernel_ms;   // the problem's time in the kernel and after it
          infos[i] = inf;
        } else if (infos) {
          rr_solve_info inf{};
          inf.status = st;
          inf.iters = out[i].iters;
          inf.op_applies = (pv[i].kind == 1 ? 3 : 1) * out[i].iters;
          inf.relres = out[i].relres;
          inf.true_relres = out[i].true_relres;
          inf.omega = pv[i].omega;
          inf.ms = kernel_ms;   // the problem's own time on its workgroup
          inf.fallback_iter = -1;
          infos[i] = inf;
        }
        if (st != RR_OK && res == RR_OK) {
          if (st == RR_ERR_NOT_CONVERGED)
            res = fail(RR_ERR_NOT_CONVERGED, "max_iter reached before the tolerance");
          else if (st == RR_ERR_BREAKDOWN)
            res = fail(RR_ERR_BREAKDOWN, "breakdown: <p,Ap> or <r,z> not positive");
          else
            res = (rr_status)st;   // a continuation's own error; its message is kept
        }
      }
    }
  }
  for (LambdaSlot* sl : used) sl->in_use--;
  return res;
}

}  // namespace

namespace rr {
rr_status get_slot_dense(rr_handle* h, double lam, LambdaSlot** out, hipStream_t s) {
  double ms = 0.0;
  return get_slot(h, h->w.X, lam, out, &ms, s);
}
}  // namespace rr

extern "C" {

const char* rr_last_error(void) { return g_last_error.c_str(); }

rr_status setup_common(const rr_csr* X, const rr_setup_opts* opts, rr_stream stream, const MemCtx& mem,
                       rr_handle** out) {
  if (!X || !out) return fail(RR_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  rr_setup_opts o;
  RR_TRY(read_opts(opts, &o));
  if (X->n_rows < 1 || X->n_cols < 1 || X->nnz < 0)
    return fail(RR_ERR_INVALID_ARG, "X: need n_rows >= 1, n_cols >= 1, nnz >= 0");
  if (X->n_rows >= (1ll << 31) - 1 || X->n_cols >= (1ll << 31) - 1 || X->nnz >= (1ll << 31) - 1 ||
      X->n_cols + X->nnz >= (1ll << 31) - 1)
    return fail(RR_ERR_INVALID_ARG, "X: sizes must fit 32-bit indices");
  if (!X->row_ptr || (X->nnz > 0 && !X->col_idx))
    return fail(RR_ERR_INVALID_ARG, "X: null row_ptr or col_idx");
  if (o.n_clusters < 0 || o.kmeans_max_iter < 0 || o.lambda_slots < 0 || o.reserve_fcg_m < 0 ||
      o.reserve_sets < 0)
    return fail(RR_ERR_INVALID_ARG, "negative option");
  rr_handle* h = new (std::nothrow) rr_handle();
  if (!h) return fail(RR_ERR_DEVICE, "out of host memory");
  h->mem = mem;
  MemScope scope(&h->mem);
  rr_status st = ws_status(h, setup_impl(X, &o, (hipStream_t)stream, h));
  if (st != RR_OK) {
    const std::string msg = g_last_error;
    (void)hipStreamSynchronize((hipStream_t)stream);
    destroy_handle(h);
    g_last_error = msg;
    return st;
  }
  *out = h;
  return RR_OK;
}

rr_status rr_setup(const rr_csr* X, const rr_setup_opts* opts, rr_stream stream, rr_handle** out) {
  g_last_error.clear();
  return setup_common(X, opts, stream, default_mem(), out);
}

rr_status rr_setup_ws(const rr_csr* X, const rr_setup_opts* opts, void* workspace, size_t ws_bytes,
                      rr_stream stream, rr_handle** out) {
  g_last_error.clear();
  if (!workspace || ws_bytes == 0) return fail(RR_ERR_INVALID_ARG, "null or empty workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(RR_ERR_INVALID_ARG, "the workspace must be 256-byte aligned");
  MemCtx m;
  m.mode = MemCtx::kBump;
  m.base = static_cast<char*>(workspace);
  m.cap = ws_bytes;
  return setup_common(X, opts, stream, m, out);
}

rr_status rr_setup_workspace_size(const rr_csr* X, const rr_setup_opts* opts, rr_stream stream,
                                  size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(RR_ERR_INVALID_ARG, "null bytes");
  *bytes = 0;
  MemCtx m;
  m.mode = MemCtx::kCount;
  rr_handle* h = nullptr;
  RR_TRY(setup_common(X, opts, stream, m, &h));
  *bytes = h->mem.used;
  (void)hipDeviceSynchronize();
  MemScope scope(&h->mem);
  destroy_handle(h);
  return RR_OK;
}

rr_status rr_setup_dense(const rr_dense* X, const rr_setup_opts* opts, rr_stream stream,
                         rr_handle** out) {
  g_last_error.clear();
  if (!X || !out) return fail(RR_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  rr_setup_opts o;
  RR_TRY(read_opts(opts, &o));
  if (o.n_clusters < 0 || o.kmeans_max_iter < 0 || o.lambda_slots < 0)
    return fail(RR_ERR_INVALID_ARG, "negative option");
  rr_handle* h = new (std::nothrow) rr_handle();
  if (!h) return fail(RR_ERR_DEVICE, "out of host memory");
  h->mem = default_mem();
  MemScope scope(&h->mem);
  const double t0 = now_ms();
  hipStream_t s = (hipStream_t)stream;
  rr_status st = RR_OK;
  if (hipGetDevice(&h->device) != hipSuccess) st = fail(RR_ERR_DEVICE, "hipGetDevice failed");
  if (st == RR_OK) st = dense_setup(h, X, &o, s);
  if (st != RR_OK) {
    const std::string msg = g_last_error;
    (void)hipStreamSynchronize(s);
    destroy_handle(h);
    g_last_error = msg;
    return st;
  }
  h->setup_ms = now_ms() - t0;
  *out = h;
  return RR_OK;
}

rr_status rr_solve_block(rr_handle* h, double lambda, int32_t nrhs, const double* rhs,
                         int64_t ld_rhs, double* w, int64_t ld_w, const rr_solve_opts* opts,
                         rr_solve_info* info, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  g_last_error.clear();
  RR_TRY(check_handle(h));
  RR_TRY(check_lambda(lambda, false));
  if (!h->dense) return fail(RR_ERR_UNSUPPORTED, "rr_solve_block takes a handle from rr_setup_dense");
  rr_solve_opts o;
  RR_TRY(read_opts(opts, &o));
  return dense_solve_block(h, lambda, nrhs, rhs, ld_rhs, w, ld_w, &o, info, (hipStream_t)stream);
}

rr_status rr_apply_operator_block(rr_handle* h, double lambda, int32_t nrhs, const double* v,
                                  int64_t ldv, double* q, int64_t ldq, int32_t precision,
                                  rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  g_last_error.clear();
  RR_TRY(check_handle(h));
  RR_TRY(check_lambda(lambda, true));
  if (!h->dense) return fail(RR_ERR_UNSUPPORTED, "rr_apply_operator_block takes a handle from rr_setup_dense");
  return dense_apply_block(h, lambda, nrhs, v, ldv, q, ldq, precision, (hipStream_t)stream);
}

rr_status rr_destroy(rr_handle* h) {
  if (!h) return RR_OK;
  (void)hipDeviceSynchronize();
  MemScope scope(&h->mem);
  destroy_handle(h);
  return RR_OK;
}

rr_status rr_get_setup_info(const rr_handle* h, rr_setup_info* info) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!info) return fail(RR_ERR_INVALID_ARG, "null info");
  rr_setup_info i{};
  i.n_rows = h->X.N;
  i.n_cols = h->X.F;
  i.nnz = h->X.nnz;
  i.n_coarse = h->FC;
  i.n_centres = h->n_centres;
  i.kmeans_iters = h->kmeans_iters;
  i.binary = h->X.binary ? 1 : 0;
  i.setup_ms = h->setup_ms;
  i.kmeans_ms = h->kmeans_ms;
  i.plan_ms = h->tune_ms;
  i.tuned_rows_div = h->tuning.div_rows;
  i.tuned_cols_div = h->tuning.div_cols;
  i.tune_cached = h->tuning.cached;
  i.dense = h->dense ? 1 : 0;
  i.eigen_sweeps = h->eig_q ? std::max(1, h->eig_sweeps) : 0;
  if (h->dense) {
    i.nnz = (int64_t)h->X.N * h->X.F;
    for (int k = 0; k < 3; ++k) i.dense_split[k] = h->dense->split_target[k];
    i.dense_split_cached = h->dense->split_cached;
  }
  *info = i;
  return RR_OK;
}

rr_status rr_get_labels(const rr_handle* h, int32_t* labels, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!labels) return fail(RR_ERR_INVALID_ARG, "null labels");
  if (h->FC == 0) return fail(RR_ERR_INVALID_ARG, "no aggregation (n_clusters = 0)");
  k_gather_int<<<cdiv(h->X.F, kBlock), kBlock, 0, (hipStream_t)stream>>>(labels, h->labels, h->finv,
                                                                        h->X.F);
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_get_centres(const rr_handle* h, int32_t* centres, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!centres) return fail(RR_ERR_INVALID_ARG, "null centres");
  if (!h->centres || h->n_centres == 0) return fail(RR_ERR_INVALID_ARG, "no k-means seeding was run");
  RR_HIP(hipMemcpyAsync(centres, h->centres, sizeof(int) * h->n_centres, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return RR_OK;
}

rr_status rr_solve(rr_handle* h, double lambda, const double* rhs, double* w,
                   const rr_solve_opts* opts, rr_solve_info* info, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  g_last_error.clear();
  RR_TRY(check_sparse(h));
  rr_solve_opts o;
  RR_TRY(read_opts(opts, &o));
  h->mem.overflow = false;
  return ws_status(h, solve_impl(h, lambda, rhs, w, &o, info, (hipStream_t)stream));
}

rr_status rr_solve_batched(int32_t nprob, rr_handle* const* handles, const double* lambdas,
                           const double* const* rhs, double* const* w, const rr_solve_opts* opts,
                           rr_solve_info* info, rr_stream stream) {
  g_last_error.clear();
  rr_solve_opts o;
  RR_TRY(read_opts(opts, &o));
  for (int i = 0; i < nprob && handles; ++i)
    if (handles[i]) handles[i]->mem.overflow = false;
  rr_status st = solve_batched_impl(nprob, handles, lambdas, rhs, w, &o, info, (hipStream_t)stream);
  for (int i = 0; st != RR_OK && i < nprob && handles; ++i) st = ws_status(handles[i], st);
  return st;
}

rr_status rr_solve_batched_noalloc(int32_t nprob, rr_handle* const* handles, const double* lambdas,
                                   const double* const* rhs, double* const* w, const rr_solve_opts* opts,
                                   rr_solve_info* info, rr_stream stream) {
  g_last_error.clear();
  rr_solve_opts o;
  RR_TRY(read_opts(opts, &o));
  if (nprob < 0) return fail(RR_ERR_INVALID_ARG, "nprob must be >= 0");
  if (nprob == 0) return RR_OK;
  if (!handles || !lambdas || !rhs || !w) return fail(RR_ERR_INVALID_ARG, "null batch array");
  if (o.x_ref || o.residual_history)
    return fail(RR_ERR_INVALID_ARG, "x_ref and residual_history are per-problem buffers: use rr_solve");
  for (int i = 0; i < nprob; ++i) {
    if (!handles[i]) return fail(RR_ERR_INVALID_ARG, "null handle in batch");
    RR_TRY(check_sparse(handles[i]));
  }
  return solve_batched_persistent(nprob, handles, lambdas, rhs, w, o, info, (hipStream_t)stream, true);
}

rr_status rr_apply_operator(rr_handle* h, double lambda, const double* v, double* Av,
                            rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  RR_TRY(check_lambda(lambda, true));
  if (!v || !Av) return fail(RR_ERR_INVALID_ARG, "null vector");
  hipStream_t s = (hipStream_t)stream;
  Work& w = h->w;
  const int F = h->X.F;
  launch_gather(w.vin, v, h->fperm, F, s);
  launch_csr(h->X, w.vin, w.u, nullptr, s);
  Epi e = base_epi(w, lambda);
  e.p = w.vin;
  e.out = w.vout;
  launch_csc(h->X, w.u, EPI_APPLY, e, nullptr, s);
  launch_gather(Av, w.vout, h->finv, F, s);
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_apply_rhs(rr_handle* h, const double* y, double* b, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  if (!y || !b) return fail(RR_ERR_INVALID_ARG, "null vector");
  Epi e{};
  e.out = h->w.vout;
  launch_csc(h->X, y, EPI_STORE, e, nullptr, (hipStream_t)stream);   // the plain X^T y, whatever the weights
  launch_gather(b, h->w.vout, h->finv, h->X.F, (hipStream_t)stream);
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_noise_rhs(rr_handle* h, double tau, double lambda, const double* y, const double* xi1,
                       const double* xi2, double* b, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  if (!y || !xi1 || !xi2 || !b) return fail(RR_ERR_INVALID_ARG, "null vector");
  if (h->X.rw) return fail(RR_ERR_UNSUPPORTED, "noise injection is built for unweighted X");
  if (!(tau > 0.0) || !(lambda > 0.0) || !std::isfinite(tau) || !std::isfinite(lambda))
    return fail(RR_ERR_INVALID_ARG, "tau and lambda must be finite and > 0");
  hipStream_t s = (hipStream_t)stream;
  double* v = nullptr;
  RR_TRY(dalloc(&v, std::max(1, h->X.N)));
  launch_noise_rhs_in(h->X.N, y, xi1, 1.0 / std::sqrt(tau), v, s);   // y + e1
  Epi e{};
  e.out = h->w.vout;
  launch_csc(h->X, v, EPI_STORE, e, nullptr, s);
  launch_gather(b, h->w.vout, h->finv, h->X.F, s);
  launch_axpy_out(h->X.F, b, xi2, std::sqrt(lambda) / tau, s);        // + e2 / tau
  RR_HIP(hipStreamSynchronize(s));
  dfree(v);
  RR_HIP(hipGetLastError());
  return RR_OK;
}

__global__ void k_check_weights(int N, const double* d, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && !(d[i] >= 0.0 && d[i] < __builtin_inf())) *bad = 1;
}

rr_status rr_set_row_weights(rr_handle* h, const double* d, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  if (!h->X.binary) return fail(RR_ERR_UNSUPPORTED, "row weights are built for 0/1 X");
  if (h->nblk > 0) return fail(RR_ERR_UNSUPPORTED, "the block smoother's blocks are built for unweighted X");
  if (h->lsw) return fail(RR_ERR_UNSUPPORTED, "row weights with least-squares interpolation are not built");
  hipStream_t s = (hipStream_t)stream;
  const int N = h->X.N, F = h->X.F;
  if (d) {
    int* flag = nullptr;
    RR_HIP(dmalloc(&flag, sizeof(int)));
    RR_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_check_weights<<<cdiv(N, kBlock), kBlock, 0, s>>>(N, d, flag);
    int bad = 0;
    RR_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
    (void)dev_free(flag);
    if (bad) return fail(RR_ERR_INVALID_ARG, "row weights must be finite and >= 0");
    if (!h->rw) RR_TRY(dalloc(&h->rw, std::max(1, N)));
    RR_HIP(hipMemcpyAsync(h->rw, d, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  }
  const double* rw = d ? h->rw : nullptr;
  h->X.rw = rw;
  h->w.X.rw = rw;
  for (Work* e : h->extra_sets) e->X.rw = rw;
  // Jacobi diagonal: c_j = sum_i d_i x_ij (0/1 X), the column pass of d
  if (rw) {
    Epi e{};
    e.out = h->colnorm;
    launch_csc(h->X, rw, EPI_STORE, e, nullptr, s);
  } else {
    k_colnorm_binary<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, h->X.col_ptr, h->colnorm);
  }
  // Gershgorin sums g = X^T D X 1
  launch_fill(h->w.x, 1.0, F, s);
  launch_csr(h->X, h->w.x, h->w.u, nullptr, s);
  {
    Epi e{};
    e.out = h->gersh;
    launch_csc(h->X, h->w.u, EPI_STORE, e, nullptr, s);
  }
  // the Galerkin coarse matrix of the weighted operator
  if (h->FC > 0) {
    if (!rw)
      RR_TRY(build_coarse_gram(h, s));
    else if (h->crow.nlayer > 0)
      RR_TRY(weighted_gram_from_labels(h, s));
    else
      RR_TRY(build_coarse_gram_valued(h, s));
    if (h->eig_q) RR_TRY(coarse_eigen(h, &h->eig_sweeps, s));
  }
  // cached per-lambda factors, weights and captured iterations no longer hold
  for (auto& sl : h->slots) {
    sl.valid = false;
    sl.lam = -1.0;
  }
  h->w.graph.reset();
  for (Work* e : h->extra_sets) e->graph.reset();
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_set_interpolation(rr_handle* h, const double* V, int32_t n_proto, double beta,
                               const int32_t* rep, double* p, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  g_last_error.clear();
  RR_TRY(check_sparse(h));
  if (h->FC == 0) return fail(RR_ERR_INVALID_ARG, "no aggregation (n_clusters = 0)");
  if (V && (n_proto < 1 || n_proto > 64))
    return fail(RR_ERR_INVALID_ARG, "n_proto must lie in [1, 64]");
  if (V && !(beta >= 0.0 && beta < __builtin_inf()))
    return fail(RR_ERR_INVALID_ARG, "beta must be finite and non-negative");
  if (h->X.rw) return fail(RR_ERR_UNSUPPORTED, "least-squares interpolation with row weights is not built");
  if (h->eig_q)
    return fail(RR_ERR_UNSUPPORTED, "the coarse eigendecomposition assumes P^T P = I");
  hipStream_t s = (hipStream_t)stream;
  // cached per-lambda factors and captured iterations no longer hold (dropped
  // first, so that a failure part-way leaves none behind)
  for (auto& sl : h->slots) {
    sl.valid = false;
    sl.lam = -1.0;
  }
  h->w.graph.reset();
  for (Work* e : h->extra_sets) e->graph.reset();
  RR_TRY(set_interpolation(h, V, n_proto, beta, rep, p, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_prototypes(rr_handle* h, int32_t n_proto, int32_t steps, uint64_t seed, double* V,
                        double* ev, rr_stream stream) {
  g_last_error.clear();
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  if (n_proto < 1 || n_proto > 64) return fail(RR_ERR_INVALID_ARG, "n_proto must be in [1, 64]");
  if (steps == 0) steps = std::max(30, 3 * n_proto);
  if (steps < n_proto || steps > 512) return fail(RR_ERR_INVALID_ARG, "steps must be in [n_proto, 512]");
  if (!V || !ev) return fail(RR_ERR_INVALID_ARG, "null V or ev");
  return ws_status(h, lanczos_prototypes(h, n_proto, steps, seed, V, ev, (hipStream_t)stream));
}

rr_status rr_apply_rows(rr_handle* h, const double* v, double* u, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  if (!v || !u) return fail(RR_ERR_INVALID_ARG, "null vector");
  hipStream_t s = (hipStream_t)stream;
  Sparse X = h->X;
  X.rw = nullptr;   // the plain product, whatever the weights
  launch_gather(h->w.x, v, h->fperm, X.F, s);
  launch_csr(X, h->w.x, u, nullptr, s);
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_coarse_eigen(rr_handle* h, double* Q, double* ev, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!h->eig_q) return fail(RR_ERR_INVALID_ARG, "the handle was set up without coarse_eigen");
  hipStream_t s = (hipStream_t)stream;
  if (Q) RR_HIP(hipMemcpyAsync(Q, h->eig_q, sizeof(double) * h->FC * h->FC, hipMemcpyDeviceToDevice, s));
  if (ev) RR_HIP(hipMemcpyAsync(ev, h->eig_v, sizeof(double) * h->FC, hipMemcpyDeviceToDevice, s));
  return RR_OK;
}

rr_status rr_apply_precond(rr_handle* h, double lambda, int32_t precond, double omega,
                           const double* r, double* z, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  RR_TRY(check_lambda(lambda, false));
  if (!r || !z) return fail(RR_ERR_INVALID_ARG, "null vector");
  if (precond < 0 || precond > 3) return fail(RR_ERR_INVALID_ARG, "unknown preconditioner");
  hipStream_t s = (hipStream_t)stream;
  Work& w = h->w;
  const int F = h->X.F;
  launch_colnorm_diag(F, h->colnorm, lambda, w.D, s);
  if (precond == PK_NONE) {
    launch_copy(z, r, F, s);
    return RR_OK;
  }
  launch_gather(w.vin, r, h->fperm, F, s);
  if (precond == PK_JACOBI) {
    launch_jacobi_apply(F, w.vin, w.D, w.vout, s);
    launch_gather(z, w.vout, h->finv, F, s);
    return RR_OK;
  }
  if (h->FC == 0) return fail(RR_ERR_INVALID_ARG, "two-level preconditioner needs a coarse level");
  LambdaSlot* sl = nullptr;
  double ms = 0.0;
  RR_TRY(get_slot(h, w.X, lambda, &sl, &ms, s));
  if (omega == 0.0) omega = sl->omega;
  if (!std::isfinite(omega) || omega < 0.0) return fail(RR_ERR_INVALID_ARG, "omega must be finite and >= 0");
  Scalars& hs = *w.sc_host;
  std::memset(&hs, 0, sizeof(Scalars));
  hs.rz = 1.0;
  RR_HIP(hipMemcpyAsync(w.sc, &hs, sizeof(Scalars), hipMemcpyHostToDevice, s));
  if (precond == PK_VCYCLE) k_smooth<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, w.vin, w.D, omega, w.e1);
  Prof pf;
  int nrz = 0;
  w.block = false;   // this call applies the point smoother, whatever the last solve used
  RR_TRY(precond_two_level(h, w, pf, 0, precond, lambda, omega, *sl, w.vin, w.vout, nullptr, &nrz, s));
  launch_gather(z, w.vout, h->finv, F, s);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_coarse_gram(rr_handle* h, double* K, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!K) return fail(RR_ERR_INVALID_ARG, "null K");
  if (h->FC == 0) return fail(RR_ERR_INVALID_ARG, "no coarse level");
  RR_HIP(hipMemcpyAsync(K, h->K, sizeof(double) * h->FC * h->FC, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return RR_OK;
}

rr_status rr_coarse_factor(rr_handle* h, double lambda, double* L, double* Ainv, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  RR_TRY(check_lambda(lambda, false));
  if (h->FC == 0) return fail(RR_ERR_INVALID_ARG, "no coarse level");
  hipStream_t s = (hipStream_t)stream;
  if (L && h->eig_q) return fail(RR_ERR_UNSUPPORTED, "a coarse_eigen handle forms no Cholesky factor");
  LambdaSlot* sl = nullptr;
  double ms = 0.0;
  RR_TRY(get_slot(h, h->w.X, lambda, &sl, &ms, s));
  const size_t bytes = sizeof(double) * h->FC * h->FC;
  if (L) RR_HIP(hipMemcpyAsync(L, sl->L, bytes, hipMemcpyDeviceToDevice, s));
  if (Ainv) RR_HIP(hipMemcpyAsync(Ainv, sl->Ainv, bytes, hipMemcpyDeviceToDevice, s));
  return RR_OK;
}

rr_status rr_mlp_init(rr_handle* h, int32_t hidden, uint64_t seed) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  if (h->FC == 0) return fail(RR_ERR_INVALID_ARG, "no coarse level");
  if (hidden < 16 || hidden > 1024) return fail(RR_ERR_INVALID_ARG, "hidden must be in [16, 1024]");
  RR_HIP(hipDeviceSynchronize());
  RR_TRY(mlp_alloc(h->mlp, h->FC + 1, hidden, h->FC, 1024));
  if (!h->mlp_scale) RR_TRY(dalloc(&h->mlp_scale, 1));
  size_t o[7];
  h->mlp.offsets(o);
  std::vector<float> p(h->mlp.nparam, 0.0f);
  uint64_t st = seed;
  const int fan_in[3] = {h->mlp.in, hidden, hidden};
  for (int layer = 0; layer < 3; ++layer) {
    const double bound = std::sqrt(6.0 / fan_in[layer]);
    for (size_t i = o[2 * layer]; i < o[2 * layer + 1]; ++i) {
      const double u = (double)(splitmix64_next(st) >> 11) * (1.0 / 9007199254740992.0);
      p[i] = (float)((2.0 * u - 1.0) * bound);
    }
  }
  return mlp_set(h->mlp, p.data(), nullptr);
}

rr_status rr_mlp_size(const rr_handle* h, int64_t* n_params, int32_t* n_in, int32_t* n_out) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!h->mlp.w) return fail(RR_ERR_INVALID_ARG, "no network (rr_mlp_init)");
  if (n_params) *n_params = (int64_t)h->mlp.nparam;
  if (n_in) *n_in = h->mlp.in;
  if (n_out) *n_out = h->mlp.out;
  return RR_OK;
}

rr_status rr_mlp_set_weights(rr_handle* h, const float* host_params) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!h->mlp.w) return fail(RR_ERR_INVALID_ARG, "no network (rr_mlp_init)");
  if (!host_params) return fail(RR_ERR_INVALID_ARG, "null parameters");
  return mlp_set(h->mlp, host_params, nullptr);
}

rr_status rr_mlp_get_weights(const rr_handle* h, float* host_params) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  if (!h->mlp.w) return fail(RR_ERR_INVALID_ARG, "no network (rr_mlp_init)");
  if (!host_params) return fail(RR_ERR_INVALID_ARG, "null parameters");
  RR_HIP(hipDeviceSynchronize());
  RR_HIP(hipMemcpy(host_params, h->mlp.w, sizeof(float) * h->mlp.nparam, hipMemcpyDeviceToHost));
  return RR_OK;
}

rr_status rr_mlp_forward(rr_handle* h, const float* in, int32_t batch, float* out, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  Mlp& n = h->mlp;
  if (!n.w) return fail(RR_ERR_INVALID_ARG, "no network (rr_mlp_init)");
  if (batch < 0 || (batch > 0 && (!in || !out))) return fail(RR_ERR_INVALID_ARG, "bad batch");
  hipStream_t s = (hipStream_t)stream;
  for (int b0 = 0; b0 < batch; b0 += n.max_batch) {
    const int bn = std::min(n.max_batch, batch - b0);
    mlp_load_inputs(n, in + (size_t)b0 * n.in, nullptr, bn, s);
    mlp_forward(n, bn, s);
    RR_HIP(hipMemcpyAsync(out + (size_t)b0 * n.out, n.y, sizeof(float) * (size_t)bn * n.out,
                          hipMemcpyDeviceToDevice, s));
  }
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_mlp_backward(rr_handle* h, const float* in, const float* dout, int32_t batch,
                          float* grads, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  Mlp& n = h->mlp;
  if (!n.w) return fail(RR_ERR_INVALID_ARG, "no network (rr_mlp_init)");
  if (batch < 1 || batch > n.max_batch || !in || !dout || !grads)
    return fail(RR_ERR_INVALID_ARG, "batch must be in [1, 1024] with non-null arrays");
  hipStream_t s = (hipStream_t)stream;
  mlp_load_inputs(n, in, nullptr, batch, s);
  mlp_forward(n, batch, s);
  mlp_set_dout(n, dout, batch, s);
  mlp_backward(n, batch, s);
  RR_HIP(hipMemcpyAsync(grads, n.g, sizeof(float) * n.nparam, hipMemcpyDeviceToDevice, s));
  RR_HIP(hipGetLastError());
  return RR_OK;
}

rr_status rr_mlp_train(rr_handle* h, const float* in, const float* target, int64_t npairs,
                       const rr_mlp_train_opts* opts, float* loss_history, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  Mlp& n = h->mlp;
  if (!n.w) return fail(RR_ERR_INVALID_ARG, "no network (rr_mlp_init)");
  if (npairs < 1 || !in || !target) return fail(RR_ERR_INVALID_ARG, "need n >= 1 pairs");
  rr_mlp_train_opts o;
  RR_TRY(read_opts(opts, &o));
  const int epochs = o.epochs > 0 ? o.epochs : 20;
  const int B = o.batch > 0 ? o.batch : 256;
  if (B > n.max_batch || npairs > (1LL << 31) - 1)
    return fail(RR_ERR_INVALID_ARG, "batch must be <= 1024 and n < 2^31");
  const float lr = o.lr > 0 ? (float)o.lr : 1e-3f;
  hipStream_t s = (hipStream_t)stream;
  const int N = (int)npairs;
  std::vector<int> order(N);
  int* d_order = nullptr;
  RR_TRY(dalloc(&d_order, N));
  std::vector<float> err(n.max_batch);
  uint64_t st = o.seed;
  rr_status res = RR_OK;
  for (int ep = 0; ep < epochs && res == RR_OK; ++ep) {
    for (int i = 0; i < N; ++i) order[i] = i;
    for (int i = N - 1; i > 0; --i) {   // Fisher-Yates with SplitMix64 draws
      const int j = (int)(splitmix64_next(st) % (uint64_t)(i + 1));
      std::swap(order[i], order[j]);
    }
    if (hipMemcpyAsync(d_order, order.data(), sizeof(int) * N, hipMemcpyHostToDevice, s) != hipSuccess) {
      res = fail(RR_ERR_DEVICE, "hipMemcpyAsync");
      break;
    }
    double tot = 0.0;
    for (int b0 = 0; b0 < N; b0 += B) {
      const int bn = std::min(B, N - b0);
      mlp_load_inputs(n, in, d_order + b0, bn, s);
      mlp_forward(n, bn, s);
      mlp_loss_grad(n, target, d_order + b0, bn, s);
      mlp_backward(n, bn, s);
      mlp_adam(n, lr, s);
      if (loss_history) {
        if (hipMemcpyAsync(err.data(), n.err2, sizeof(float) * bn, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
          res = fail(RR_ERR_DEVICE, "loss readback");
          break;
        }
        for (int i = 0; i < bn; ++i) tot += err[i];
      }
    }
    if (loss_history) loss_history[ep] = (float)(0.5 * tot / N);
  }
  (void)hipStreamSynchronize(s);
  dfree(d_order);
  RR_TRY(res);
  RR_HIP(hipGetLastError());
  return RR_OK;
}

namespace {
// Pairs from solves driven by the algebraic cycle (V(1,1) PCG) or, with
// `learned`, by the network itself (its flexible-CG solve, which visits the
// residuals the network's own corrections leave).
rr_status collect_pairs(rr_handle* h, bool learned, const double* lambdas, int32_t n_solves,
                        int32_t pairs_per_solve, int32_t every, const double* y, float* inputs,
                        float* targets, int64_t* n_pairs, rr_stream stream) {
  if (h->FC == 0) return fail(RR_ERR_INVALID_ARG, "no coarse level");
  if (n_solves < 0 || pairs_per_solve < 1 || every < 1 || !lambdas || !y || !inputs || !targets)
    return fail(RR_ERR_INVALID_ARG, "bad pair-collection arguments");
  hipStream_t s = (hipStream_t)stream;
  const int FC = h->FC;
  double* snap = nullptr;
  double* ainv_rc = nullptr;
  RR_TRY(dalloc(&snap, (size_t)pairs_per_solve * FC));
  RR_TRY(dalloc(&ainv_rc, (size_t)pairs_per_solve * FC));
  double* wtmp = nullptr;
  RR_TRY(dalloc(&wtmp, h->X.F));
  int64_t written = 0;
  rr_status res = RR_OK;
  for (int i = 0; i < n_solves && res == RR_OK; ++i) {
    Solve sv;
    sv.h = h;
    sv.ws = &h->w;
    sv.lam = lambdas[i];
    sv.rhs = y;
    sv.wout = wtmp;
    sv.op.precond = learned ? PK_LEARNED : PK_VCYCLE;
    if (learned) {
      sv.op.krylov = RR_KRYLOV_FCG;
      sv.op.fcg_m = 4;
    }
    sv.op.tol = 1e-10;
    sv.op.max_iter = every * pairs_per_solve;
    sv.s = s;
    sv.snap = snap;
    sv.snap_every = every;
    sv.snap_max = pairs_per_solve;
    res = sv.begin();
    while (res == RR_OK && !sv.done) {
      res = sv.queue_chunk();
      if (res == RR_OK) res = sv.poll();
    }
    rr_solve_info inf{};
    if (res == RR_OK) {
      const rr_status fs = sv.finish(&inf);
      if (fs != RR_OK && fs != RR_ERR_NOT_CONVERGED) res = fs;
      g_last_error.clear();
    }
    if (res == RR_OK) {
      // the cycle after the last update does not run: its snapshot is stale
      const int valid = std::min(pairs_per_solve, std::max(0, inf.iters - 1) / every);
      for (int q = 0; q < valid; ++q)
        launch_gemv(FC, sv.sl->Ainv, snap + (size_t)q * FC, ainv_rc + (size_t)q * FC, nullptr, s);
      launch_make_pairs(FC, valid, snap, ainv_rc, h->K, lambdas[i], inputs + (size_t)written * (FC + 1),
                        targets + (size_t)written * FC, s);
      written += valid;
      if (hipStreamSynchronize(s) != hipSuccess) res = fail(RR_ERR_DEVICE, "pair construction");
    }
    sv.release();
  }
  (void)hipStreamSynchronize(s);
  dfree(snap);
  dfree(ainv_rc);
  dfree(wtmp);
  RR_TRY(res);
  if (n_pairs) *n_pairs = written;
  return RR_OK;
}
}  // namespace

rr_status rr_collect_pairs(rr_handle* h, const double* lambdas, int32_t n_solves,
                           int32_t pairs_per_solve, int32_t every, const double* y, float* inputs,
                           float* targets, int64_t* n_pairs, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  return collect_pairs(h, false, lambdas, n_solves, pairs_per_solve, every, y, inputs, targets, n_pairs,
                       stream);
}

rr_status rr_collect_pairs_learned(rr_handle* h, const double* lambdas, int32_t n_solves,
                                   int32_t pairs_per_solve, int32_t every, const double* y, float* inputs,
                                   float* targets, int64_t* n_pairs, rr_stream stream) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_sparse(h));
  if (!h->mlp.w || h->mlp.in != h->FC + 1 || h->mlp.out != h->FC)
    return fail(RR_ERR_INVALID_ARG, "no network for this coarse level (rr_mlp_init)");
  return collect_pairs(h, true, lambdas, n_solves, pairs_per_solve, every, y, inputs, targets, n_pairs,
                       stream);
}

rr_status rr_smoother_weight(rr_handle* h, double lambda, double* omega) {
  MemScope mem_scope_(mem_of(h));
  RR_TRY(check_handle(h));
  RR_TRY(check_lambda(lambda, false));
  if (!omega) return fail(RR_ERR_INVALID_ARG, "null omega");
  return auto_omega(h, h->w.X, lambda, omega, nullptr);
}

}  // extern "C"
