// Internal declarations shared by the HIP translation units of librr.
// Nothing here is part of the C ABI (include/rr.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rr.h"

namespace rr {

constexpr int kBlock = 256;          // threads per block for streaming kernels
constexpr int kMergeItems = 8;       // merge-path items per thread
constexpr int kMergeTile = kBlock * kMergeItems;

// Device-resident Krylov state.  Reduction kernels finish their scalar in the
// last block to arrive (integer ticket), so the host never reads a scalar
// inside the iteration.
struct Scalars {
  double rz;        // <r, z> of the current iterate
  double pq;        // <p, A p>
  double alpha, beta;
  double rr;        // ||r||^2
  double bb;        // ||b||^2
  double ee;        // ||x - x_ref||^2
  double ref2;      // ||x_ref||^2
  double tol2;      // tol^2 ||b||^2
  double errtol2;   // err_tol^2 ||x_ref||^2
  double true_rr;   // ||b - A x||^2 at exit
  double pad;
  int iter, done, status, limit;
  int fixed, use_err, pad0, pad1;
  unsigned int ticket;
  unsigned int pad2[15];
};

// Epilogue arguments of the CSC (column-segment) reduction.
enum EpiMode {
  EPI_STORE = 0,      // out[s] = t
  EPI_APPLY = 1,      // out[s] = t + lam p[s]
  EPI_APPLY_DOT = 2,  // q = t + lam p[s]; out = q; <p,q> -> pq, alpha
  EPI_RESID = 3,      // out[s] = r[s] - (t + lam p[s])
  EPI_POST = 4,       // rho = r - (t + lam e2); z = e2 + w rho / D; <r,z> -> beta
  EPI_TRUE = 5,       // res = r - (t + lam x); <res,res> -> true_rr
  EPI_SCALE = 6       // out[s] = t * scale[s]
};

struct Epi {
  double lam;
  double omega;
  const double* p;      // the vector multiplied by lambda (p, e1, e2, x)
  const double* r;      // r or b
  const double* D;      // Jacobi diagonal
  const double* scale;  // per-segment scale
  double* out;
  Scalars* sc;
  double* partials;
  double* history;
};

// Merge-path plan of a segmented gather-sum out[s] = sum_{e in seg s} v[idx[e]].
struct MergePlan {
  int nseg = 0, nnz = 0, nblocks = 0, nspan = 0;
  int2* coord = nullptr;   // device [nblocks+1]: (segment, element) at each tile start
  int4* span = nullptr;    // device [nspan]: (segment, first block, last block, 0)
  double* head = nullptr;  // device [nblocks]
  double* tail = nullptr;  // device [nblocks]
};

// Sparse matrix stored both ways.
struct Sparse {
  int N = 0, F = 0, nnz = 0;
  bool binary = true;
  int* row_ptr = nullptr;   // [N+1]
  int* col_idx = nullptr;   // [nnz]
  double* val = nullptr;    // [nnz] or null
  int* col_ptr = nullptr;   // [F+1]
  int* row_idx = nullptr;   // [nnz]
  double* cval = nullptr;   // [nnz] or null (CSC order)
  int csr_group = 16;       // lanes per row in the CSR kernel
  MergePlan csc_plan;       // segments = columns
};

struct LambdaSlot {
  double lam = -1.0;
  double* L = nullptr;      // [FC*FC] lower Cholesky factor
  double* Ainv = nullptr;   // [FC*FC]
  double omega = 0.0;       // automatic smoother weight at this lambda
  bool valid = false;
  unsigned long long stamp = 0;
};

struct Work {
  double *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
  double *e1 = nullptr, *e2 = nullptr, *rho = nullptr, *b = nullptr;
  double *D = nullptr;            // Jacobi diagonal at the current lambda
  double *vin = nullptr, *vout = nullptr, *xref = nullptr;  // boundary permutation buffers
  double *u = nullptr;            // [N]
  double *c = nullptr, *yc = nullptr;   // [FC]
  double *partials = nullptr;     // reduction partials
  int npartials = 0;
  Scalars* sc = nullptr;
  Scalars* sc_host = nullptr;     // pinned mirror
};

}  // namespace rr

struct rr_handle {
  int device = 0;
  rr::Sparse X;
  int* fperm = nullptr;         // [F] internal feature -> caller's feature
  int* finv = nullptr;          // [F] caller's feature -> internal feature
  double* colnorm = nullptr;    // [F] ||x_j||^2
  double* gersh = nullptr;      // [F] (X^T X 1)_j
  bool nonneg = true;
  // aggregation
  int k_req = 0, FC = 0, n_centres = 0, kmeans_iters = 0;
  int* labels = nullptr;        // [F] in [0, FC)
  int* centres = nullptr;       // [k] caller's feature indices, draw order
  int* csize = nullptr;         // [FC]
  double* cscale = nullptr;     // [FC] 1/sqrt(n_s)
  int* perm = nullptr;          // [F] features sorted by cluster (stable)
  int* coff = nullptr;          // [FC+1] cluster offsets into perm
  rr::MergePlan restrict_plan;  // segments = clusters over perm
  double* K = nullptr;          // [FC*FC] coarse Gram
  std::vector<rr::LambdaSlot> slots;
  unsigned long long stamp = 0;
  double* chol_work = nullptr;  // [FC*FC] scratch for the factorization
  int* chol_flag = nullptr;     // device int
  rr::Work w;
  double setup_ms = 0, kmeans_ms = 0;
  std::vector<hipEvent_t> ev_pool;
};

namespace rr {

// ---- error reporting -------------------------------------------------------
void set_error(const std::string& msg);
rr_status fail(rr_status st, const std::string& msg);

#define RR_HIP(call)                                                         \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::rr::fail(RR_ERR_DEVICE, std::string(#call) + ": " +          \
                                           hipGetErrorString(e_));           \
  } while (0)

#define RR_TRY(call)                                                         \
  do {                                                                       \
    rr_status s_ = (call);                                                   \
    if (s_ != RR_OK) return s_;                                              \
  } while (0)

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// ---- sparse kernels (spmv.hip) ----------------------------------------------
rr_status build_merge_plan(MergePlan& mp, const int* d_seg_end, const int* d_seg_ptr,
                           int nseg, int nnz, hipStream_t s);
void free_merge_plan(MergePlan& mp);
// u = X v (CSR).  done may be null.
void launch_csr(const Sparse& X, const double* v, double* u, const int* done, hipStream_t s);
// Column-segment reduction t_s = sum_e v[idx[e]] (* val[e]) with epilogue `mode`.
void launch_segsum(const MergePlan& mp, const int* seg_end, const int* idx, const double* val,
                   const double* v, int mode, const Epi& e, const int* done, hipStream_t s);
// X^T u with epilogue, using the CSC of X.
void launch_csc(const Sparse& X, const double* u, int mode, const Epi& e, const int* done,
                hipStream_t s);
rr_status build_csc(Sparse& X, hipStream_t s);
rr_status renumber_features(Sparse& X, int* fperm, int* finv, hipStream_t s);
rr_status validate_csr(const Sparse& X, hipStream_t s);

// ---- vector kernels (blas1.hip) ---------------------------------------------
enum PcgKind { PK_NONE = 0, PK_JACOBI = 1, PK_VCYCLE = 2, PK_ADDITIVE = 3 };
void launch_pcg_init(int F, const double* b, double* x, double* r, double* p, double* z,
                     double* e1, const double* D, const double* xref, double omega, int kind,
                     Scalars* sc, double* partials, double* history, hipStream_t s);
void launch_pcg_update(int F, double* x, double* r, const double* p, const double* q,
                       double* z, double* e1, const double* D, const double* xref,
                       double omega, int kind, Scalars* sc, double* partials, double* history,
                       hipStream_t s);
void launch_pupdate(int F, double* p, const double* z, Scalars* sc, hipStream_t s);
void launch_prolong(int F, const int* labels, const double* cscale, const double* yc,
                    const double* e1, double* out, const double* r, const double* D,
                    double omega, int additive, Scalars* sc, double* partials, hipStream_t s);
void launch_fill(double* x, double v, long long n, hipStream_t s);
// dst[i] = src[idx[i]]
void launch_gather(double* dst, const double* src, const int* idx, int n, hipStream_t s);
void launch_copy(double* dst, const double* src, long long n, hipStream_t s);
void launch_colnorm_diag(int F, const double* colnorm, double lam, double* D, hipStream_t s);
void launch_jacobi_apply(int F, const double* r, const double* D, double* z, hipStream_t s);
void launch_omega_gersh(int F, const double* g, const double* colnorm, double lam,
                        double* out, double* partials, unsigned* ticket, hipStream_t s);
void launch_axpby(long long n, double a, const double* x, double b, double* y,
                  hipStream_t s);
void launch_dot(long long n, const double* x, const double* y, double* out,
                double* partials, unsigned* ticket, hipStream_t s);
void launch_gemv(int n, const double* A, const double* x, double* y, const int* done,
                 hipStream_t s);

// ---- coarse level (coarse.hip) ---------------------------------------------
rr_status coarse_factor(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s);

// ---- clustering (kmeans.hip) -----------------------------------------------
rr_status run_kmeans(rr_handle* h, int k, uint64_t seed, int max_iter, hipStream_t s);
rr_status set_labels(rr_handle* h, const int* labels_in, int nlab, hipStream_t s);
rr_status build_coarse_gram(rr_handle* h, hipStream_t s);

}  // namespace rr
