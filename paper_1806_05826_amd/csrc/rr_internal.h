// Internal declarations shared by the HIP translation units of librr.
// Nothing here is part of the C ABI (include/rr.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <deque>
#include <string>
#include <vector>

#include "../../include/rr.h"

namespace rr {

// ---- device memory (alloc.hip) ---------------------------------------------
// The memory context of a handle: where its device allocations come from.
struct MemCtx {
  enum Mode { kHip = 0, kHook = 1, kBump = 2, kCount = 3 };
  Mode mode = kHip;
  rr_alloc_fn alloc = nullptr;   // kHook: the caller's allocator
  rr_free_fn free = nullptr;
  void* ctx = nullptr;
  char* base = nullptr;          // kBump: the caller's workspace
  size_t cap = 0;
  size_t used = 0;               // kBump / kCount: arena bytes taken
  bool overflow = false;         // kBump: a request did not fit
};
// Makes m the calling thread's memory context for the scope's lifetime.
class MemScope {
 public:
  explicit MemScope(MemCtx* m);
  ~MemScope();
  MemScope(const MemScope&) = delete;
  MemScope& operator=(const MemScope&) = delete;
 private:
  MemCtx* saved_;
};
MemCtx default_mem();   // the caller's allocator when installed, else hipMalloc
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t dev_free(void* p);
template <typename T>
inline hipError_t dmalloc(T** p, size_t bytes) {
  return dev_malloc(reinterpret_cast<void**>(p), bytes);
}


constexpr int kBlock = 256;          // threads per block for streaming kernels
constexpr int kMergeItems = 8;       // merge-path items per thread
constexpr int kMergeTile = kBlock * kMergeItems;

// Device-resident Krylov state.  A scalar is written by block 0 of the kernel
// that forms it and read by later kernels only, so the host never reads a
// scalar inside the iteration.
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
  double rz_next;   // <r, z> of the newest residual, consumed by the next update
  double pad3;
  int iter, done, status, limit;
  int fixed, use_err, pad0, pad1;
  unsigned int pad2[16];
};

// Block partials of the solver's reductions.  A producer kernel stores one
// value per block (plain stores); every block of the consuming kernel adds
// them in the same order, so all blocks see the same scalar without atomics.
constexpr int kMaxParts = 1024;         // partials a consumer block adds itself
constexpr int kMaxReduceBlocks = 4096;  // grid cap of the SELL segment reduction
struct Parts {
  double* pq = nullptr;    // <p, Ap>            [n_red]
  double* upd = nullptr;   // ||r||^2, err^2, <r,z> (Jacobi/CG)   [3 * n_vec]
  double* rz = nullptr;    // <r, z> from the preconditioner      [n_red or n_vec]
  double* init = nullptr;  // ||b||^2, ||x_ref||^2, <r,z>          [3 * n_vec]
  double* tr = nullptr;    // ||b - Ax||^2                         [n_red]
  double* dots = nullptr;  // flexible CG: <z, A p_k>               [kMaxFcg * n_vec]
  int n_red = 0;           // blocks of the column reduction (CSC epilogue)
  int n_vec = 0;           // blocks of the vector kernels
};

// What the kernel after the x/r update checks before doing its own work.
struct StageArgs {
  Scalars* sc;
  const double* upd;       // update partials (3 * n)
  int n;
  double* history;
  int kind;
};

// The PCG direction update p = z + beta p folded into the next iteration:
// beta = <r,z>_new / sc->rz (0 while sc->rz is 0: the first direction), with
// <r,z>_new the sum of parts[0, n).  The row pass forms X p = X z + beta X p
// (launch_rows_pupd, X p of the previous direction kept in its output), and
// the column reduction that follows (EPI_APPLY_DOT_P) writes p itself.
struct PUpd {
  const double* parts;
  int n;
  Scalars* sc;
};

// Window of previous directions of flexible CG (oldest first).
constexpr int kMaxFcg = 16;
// Internal status of a learned-correction solve whose flexible-CG step met a
// non-finite or non-positive <p, A p> or a non-finite <p, r>: the host
// switches the solve to the algebraic V(1,1) cycle and restarts the
// flexible-CG history (never returned through the ABI).
constexpr int kStatusFallback = 100;
struct FcgWindow {
  const double* p[kMaxFcg];
  const double* ap[kMaxFcg];
  int slot[kMaxFcg];        // ring slot of each direction (its <p, Ap>)
  int n;
};

// Epilogue arguments of the CSC (column-segment) reduction.
enum EpiMode {
  EPI_STORE = 0,      // out[s] = t
  EPI_APPLY = 1,      // out[s] = t + lam p[s]
  EPI_APPLY_DOT = 2,  // q = t + lam p[s]; out = q; <p,q> -> pq, alpha
  EPI_RESID = 3,      // out[s] = r[s] - (t + lam p[s])
  EPI_POST = 4,       // rho = r - (t + lam e2); z = e2 + w rho / D; <r,z> -> beta
  EPI_TRUE = 5,       // res = r - (t + lam x); <res,res> -> true_rr
  EPI_SCALE = 6,      // out[s] = t * scale[s]
  EPI_POST_P = 7,     // EPI_POST with e2 = e1 + P yc formed in place (p = e1)
  EPI_APPLY_DOT_P = 8 // p = z + beta p (z in r, beta in sc, written to pnew), then EPI_APPLY_DOT
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
  double* partials;      // block partials of the epilogue's dot product
  double* history;
  const int* labels;     // EPI_POST_P: cluster of every feature,
  const double* cscale;  // the prolongation's 1/sqrt(n_s)
  const double* yc;      // and the coarse correction
  const int* opos;       // EPI_RESID: store segment s at opos[s] (cluster order), or at s
  // restriction from the row pass (k_seg1 with XP): cluster s subtracts its
  // pieces xpart[xpos[q]], q in [xbase[s], xbase[s+1]), the partial sums of
  // (X P)^T u over (cluster, row slice) pairs
  const int* xbase;
  const int* xpos;
  const double* xpart;
  double* pnew;          // EPI_APPLY_DOT_P: where the updated direction goes (p itself)
};

// Single-precision vectors of an inner solve of iterative refinement.
struct IrVectors {
  float *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
  float *e1 = nullptr, *e2 = nullptr, *D = nullptr;   // [F]
  float* u = nullptr;                                                  // [N]
  float* part_cols = nullptr;   // column pass partial sums (sliced pass)
};

// The learned coarse correction's network (mlp.hip).
struct Mlp {
  int in = 0, hid = 0, out = 0, max_batch = 0, t = 0;
  size_t nparam = 0;
  float* w = nullptr;        // FP32 master parameters W1 b1 W2 b2 W3 b3
  uint16_t* w16 = nullptr;   // BF16 copy (the products' operands)
  float *m = nullptr, *v = nullptr, *g = nullptr;   // Adam moments, gradient
  uint16_t* xb = nullptr;    // [max_batch, in] BF16 inputs
  float *z1 = nullptr, *z2 = nullptr, *y = nullptr;          // pre-activations, output
  uint16_t *a1 = nullptr, *a2 = nullptr;                     // BF16 activations
  float *dy32 = nullptr, *dz2 = nullptr, *dz1 = nullptr;     // FP32 backward signals
  uint16_t *dy16 = nullptr, *dz2b = nullptr, *dz1b = nullptr;
  float* err2 = nullptr;     // per-row squared errors
  int* rows = nullptr;       // mini-batch row indices
  void offsets(size_t* o) const;   // o[0..6]: W1 b1 W2 b2 W3 b3 end
};

// Epilogue arguments of the single-precision column reduction.
struct Epi32 {
  double lam;
  double omega;
  const float* p;
  const float* r;
  const float* D;
  float* out;
  double* out64;      // EPI_RESID: FP64 result
  double* partials;
};

// Merge-path plan of a segmented gather-sum out[s] = sum_{e in seg s} v[idx[e]].
struct MergePlan {
  int nseg = 0, nnz = 0, nblocks = 0, nspan = 0;
  int2* coord = nullptr;   // device [nblocks+1]: (segment, element) at each tile start
  int4* span = nullptr;    // device [nspan]: (segment, first block, last block, 0)
  double* head = nullptr;  // device [nblocks]
  double* tail = nullptr;  // device [nblocks]
  // wave-item form for sums without a dot product (the restriction, built
  // by build_chunk_plan): witem (segment, first, end, chunk slot or -1), a
  // segment of up to kWaveSeg entries per item, longer ones in chunks whose
  // sums go to cpart; fitem (segment, first slot, chunks, 0) finishes those
  int nwitem = 0, nfitem = 0, ncpart = 0;
  int4* witem = nullptr;
  int4* fitem = nullptr;
  double* cpart = nullptr;   // device [ncpart] (each work set holds its own)
};

// Sliced-ELL plan of a segmented gather-sum out_s = sum_{e in s} v[g_e]
// (see sell.hip).  The gathered vector is cut into slices of W entries that
// live in LDS.
constexpr int kSliceRows = 16384;     // W: 128 KB of FP64 per slice in LDS
constexpr int kSliceBlock = 1024;     // threads per sliced workgroup
constexpr int kSliceWaves = kSliceBlock / 64;
struct SellPlan {
  int S = 0, gdim = 0, W = 0, R = 0, nblk = 0, ntask = 0, nslots = 0, nitems = 0, nout = 0;
  int pass = 0;               // 0: rows of X (u = X v), 1: columns (t = X^T u)
  long long idx_bytes = 0;
  uint16_t* idx = nullptr;    // packed local indexes (bit 15: last entry of a pair)
  int4* task = nullptr;       // [ntask]
  int* wrange = nullptr;      // [nblk * (kSliceWaves + 1)] task range of every wave
  int* bslice = nullptr;      // [nblk] slice of every workgroup
  int* pos = nullptr;         // [nitems] output position of every piece of a (segment, slice) pair
  int* sbase = nullptr;       // [S+1] first piece of every segment
  int* lseg = nullptr;        // [nlong] segments of more than 16 pieces (added by a wave each)
  int nlong = 0;
  double* part = nullptr;     // [nout] partial sums
  double* val = nullptr;      // valued X: the entries' values beside idx (0 for padding)
};

// Row pass of 0/1 X without partial sums (rows.hip): layer c of 64 / L rows
// holds lane-interleaved hot uint16 indexes into the LDS copy of v[0, W) and
// cold int32 feature indexes gathered from global memory.
struct RowPlan {
  int N = 0, F = 0, W = 0, L = 1, nlayer = 0, nblk = 0;
  long long hot_entries = 0, cold_entries = 0, idx_bytes = 0;
  int4* layer = nullptr;      // [nlayer] (hot offset, hot length, cold offset, cold length) per lane
  uint16_t* hidx = nullptr;   // hot lane streams (W = the zero entry)
  int* cidx = nullptr;        // cold lane streams (-1 = padding)
  double* hval = nullptr;     // valued X: the entries' values beside hidx (0 for padding)
  double* cval = nullptr;     // valued X: the entries' values beside cidx (0 for padding)
};

// Persistent batched solver (batch.hip): problems of at most kBatchFMax
// features, rows in chunks of kBatchRows staged through LDS.
constexpr int kBatchFMax = 8192;
constexpr int kBatchRows = 10240;

// Per-handle plan of the batched solver (0/1 X, F <= kBatchFMax).
struct BatchPlan {
  int nchunk = 0, grow = 1;   // row chunks; lanes per row
  int cls[3] = {0, 0, 0};     // column classes: [0, cls0) 64 lanes, then 16, 4, 1
  int* csplit = nullptr;      // [(nchunk + 1) * F] CSC entry of column j at chunk h's first row
  uint16_t* ci16 = nullptr;   // [nnz] CSR column indices (F <= 8192)
  uint16_t* ri16 = nullptr;   // [nnz] CSC row indices less their chunk's first row
  int tuned = 0;              // grow: 0 from the rows' length, 1 timed here, 2 from the tuning cache
};

// One problem of a persistent batched solve (device descriptor).
struct BatchProb {
  int N, F, FC, nchunk, grow, kind, rhs_is_b, max_iter, fixed;
  int cap;   // > 0: leave the kernel at this iteration (the host continues the solve)
  int cls[3];
  const int *rp, *csplit, *perm, *coff, *labels, *fperm, *finv;
  const uint16_t *ci, *ri;
  const double *cscale, *Ainv, *colnorm, *rhs;
  double lam, omega, tol2;
  double *w, *x, *r, *p, *z, *e1, *b, *t;
};
// status kStatusYield: the problem left at iteration `iters` with x, r, p
// in its work set and <r,z> = rz, ||b||^2 = bb
constexpr int kStatusYield = 101;
struct BatchOut {
  int status, iters;
  double relres, true_relres;
  double rz, bb;
  long long t_begin, t_end;   // wall_clock64() around the problem's solve
};
// The allocation-free persistent solve's buffers, in the library's static
// device scratch of this GPU (batch.hip).
constexpr int kStaticProblems = 2048;
struct BatchScratch {
  BatchProb* probs = nullptr;
  int* order = nullptr;
  BatchOut* out = nullptr;
  int* queue = nullptr;
  int cap = 0;
};

// Autotuning record of the operator plans (see build_sell_plans): lanes per
// row of the row pass (div_rows) and the column pass's lane-stream divisor.
struct SellTuning {
  int div_rows = 2, div_cols = 2, cached = 0, n = 0;
  int cand_div[8] = {}, cand_pass[8] = {};
  float cand_ms[8] = {};
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
  const double* rw = nullptr;   // [N] row weights d (rr_set_row_weights): the row pass
                                // forms u = D X v, so the operator is X^T D X + lam I
  int csr_group = 16;       // lanes per row in the CSR kernel
  MergePlan csc_plan;       // segments = columns (merge-path form, valued X)
  RowPlan rows;             // u = X v   (0/1 X)
  SellPlan sell_csc;        // t = X^T u (0/1 X)
  BatchPlan bplan;          // persistent batched solver (0/1 X, F <= kBatchFMax)
  bool sliced = false;      // rows and sell_csc built: the operator runs the sliced passes
  int num_cu = 256;
};

struct LambdaSlot {
  double lam = -1.0;
  double* L = nullptr;      // [FC*FC] lower Cholesky factor
  double* Ainv = nullptr;   // [FC*FC]
  double omega = 0.0;       // automatic smoother weight at this lambda
  double* Dinv = nullptr;   // block smoother: (X_B^T X_B + lam I)^-1, 32 x 32 per block
  double omega_block = 0.0; // its automatic weight (0: not yet estimated)
  bool valid = false;
  unsigned long long stamp = 0;
  int in_use = 0;           // solves running with this factor (not evicted meanwhile)
};

// A captured chunk of PCG iterations and what its launches depend on.
struct GraphKey {
  int kind = -1;
  double lam = 0.0, omega = 0.0;
  const double* ainv = nullptr;
  const double* xref = nullptr;
  const double* history = nullptr;
  int chunk = 0;
  const double* dinv = nullptr;   // block smoother's inverses (null: point smoother)
  bool cycle32 = false;           // the preconditioner's cycle in FP32
  int pu_n = -1;                  // direction update folded into the next iteration: its partials
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && lam == o.lam && omega == o.omega && ainv == o.ainv &&
           xref == o.xref && history == o.history && chunk == o.chunk && dinv == o.dinv &&
           cycle32 == o.cycle32 && pu_n == o.pu_n;
  }
};
struct ChunkGraph {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev = nullptr;        // orders replays on the set's stream with the caller's
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key = GraphKey{};
  }
};

struct Work {
  double *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
  double *e1 = nullptr, *e2 = nullptr, *rho = nullptr, *b = nullptr;
  double *D = nullptr;            // Jacobi diagonal at the current lambda
  double *vin = nullptr, *vout = nullptr, *xref = nullptr;  // boundary permutation buffers
  double *u = nullptr;            // [N]
  double *up = nullptr;           // [N] X p of the current direction (folded direction update)
  double *c = nullptr, *yc = nullptr;   // [FC]
  double *partials = nullptr;     // reduction partials
  int npartials = 0;
  Parts parts;
  int fcg_m = 0;                  // ring size of the flexible-CG directions
  double *fcg_p = nullptr, *fcg_ap = nullptr, *fcg_paps = nullptr;   // [m F], [m F], [m]
  Scalars* sc = nullptr;
  Scalars* sc_host = nullptr;     // pinned mirror
  // The matrix and restriction plans as this set sees them: the handle's
  // plans with this set's own partial-sum buffers, so that solves on
  // different sets of one handle can run at the same time.
  Sparse X;
  MergePlan rplan;
  double* xp_part = nullptr;      // partial sums of the X P column pass (this set's own)
  MergePlan xr;                   // the X P restriction's items with this set's chunk sums
  bool extra = false;             // an additional set (owns those buffers)
  bool block = false;             // the running solve smooths with the block smoother
  int rsteps = 2;                 // CG steps of the rougher (RR_PRECOND_ROUGHER)
  bool rjacobi = false;           // Jacobi-preconditioned rougher steps
  IrVectors f32;                  // single-precision vectors, allocated on first use
  ChunkGraph graph;               // captured PCG chunk (rr_solve_opts.graph)
  hipStream_t stream = nullptr;   // batched solves: this set's stream
};

// Dense X (rr_setup_dense).  Four resident copies, FP32 and BF16, row-major
// and transposed, so that both products of the operator stream their first
// operand along the contraction index; rows and columns are zero-padded to
// multiples of kDensePad.
constexpr int kDensePad = 128;
struct DenseX {
  int N = 0, F = 0, Np = 0, Fp = 0;
  float* X32 = nullptr;       // [Np x Fp] row-major
  float* XT32 = nullptr;      // [Fp x Np] row-major
  uint16_t* Xb = nullptr;     // BF16 of X32
  uint16_t* XTb = nullptr;    // BF16 of XT32
  double* Xc = nullptr;       // [FC x Np] coarse columns X P (row s = column s of X P)
  // workgroups the column pass's split contraction aims at, per operator
  // precision (FP64, BF16, FP32); chosen by timing when the setup asks
  int split_target[3] = {1024, 256, 1024};
  int split_cached = 0;       // 1: the targets came from an earlier measurement
};

// Buffers of a block solve with up to m_cap right-hand sides.  F-blocks are
// column-major with leading dimension Fp, N-blocks with Np; rows past F (N)
// and columns past the solve's m are never written after the zero fill.
struct DenseWork {
  int m_cap = 0, nb = 0;      // nb = column partials per F-vector (blocks of 1024)
  double *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
  double *e1 = nullptr, *e2 = nullptr, *rho = nullptr, *b = nullptr;
  double *wx = nullptr, *wr = nullptr;  // refinement: FP64 iterate and residual
  double* D = nullptr;        // [Fp] Jacobi diagonal
  uint16_t* vb = nullptr;     // BF16 copy of the operator's input block
  uint16_t* ub = nullptr;     // BF16 U = X V  [Np x m_cap]
  double* u = nullptr;        // FP64 U        [Np x m_cap]
  float* uf = nullptr;        // FP32 U        [Np x m_cap]
  void* part = nullptr;       // split-K partial sums
  size_t part_bytes = 0;
  double *c = nullptr, *yc = nullptr;   // coarse blocks [FC x m_cap]
  double* parts = nullptr;    // column partials: 6 regions of [m_cap x nb]
  double *rz = nullptr, *pq = nullptr, *alpha = nullptr, *beta = nullptr;
  double *rr = nullptr, *bb = nullptr;  // per column
  int *done = nullptr, *iters = nullptr, *status = nullptr;  // per column
  int* done_in = nullptr;     // per column: finished before a solve starts
  int* nactive = nullptr;     // device int: columns still iterating
  int* nactive_host = nullptr;  // pinned mirror
};

}  // namespace rr

// X's rows with every column index replaced by its cluster label, for the
// V(1,1) cycle's second row pass (see crows.hip); 0/1 X only.
constexpr int kMaxCrClusters = 8191;   // F_C + 1 FP64 entries in 64 KB of LDS
struct ClusterRows {
  int nlayer = 0;
  int2* layer = nullptr;      // [nlayer] (first entry, entries per lane)
  uint16_t* ent = nullptr;    // labels, lane-interleaved in groups of 4
  int* rowid = nullptr;       // [nlayer * 64] row of every lane, -1 for none
};

struct rr_handle {
  int device = 0;
  rr::MemCtx mem;               // where the handle's device memory comes from
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
  int* cpos = nullptr;          // [F] inverse of perm: feature j sits at cpos[j]
  int* coff = nullptr;          // [FC+1] cluster offsets into perm
  rr::MergePlan restrict_plan;  // segments = clusters over perm
  ClusterRows crow;             // label table for the V(1,1) second row pass
  rr::SellPlan xp;              // X's entries by cluster: column pass of X P (V(1,1) restriction)
  rr::MergePlan xp_restrict;    // the restriction's wave items with xp (build_xp_restrict)
  double* K = nullptr;          // [FC*FC] coarse Gram
  double* rw = nullptr;         // [N] row weights (owned), null when unweighted
  double* wxc = nullptr;        // [FCp x Np] D^1/2 X P as rows, for the weighted coarse matrix
  double* eig_q = nullptr;      // [FC*FC] eigenvectors of K (columns), with coarse_eigen
  double* eig_v = nullptr;      // [FC] their eigenvalues
  int eig_sweeps = 0;           // Jacobi sweeps the decomposition took
  // least-squares interpolation: P(j, labels[j]) = lsw[j] instead of cscale
  double* lsw = nullptr;        // [F] null: the adjusted square-root average
  double* lsw_perm = nullptr;   // [F] lsw in perm order (restriction values)
  double* pgram = nullptr;      // [FC] diagonal of P^T P
  std::deque<rr::LambdaSlot> slots;
  unsigned long long stamp = 0;
  double* chol_work = nullptr;  // [FC*FC] scratch for the factorization
  int* chol_flag = nullptr;     // device int
  rr::Mlp mlp;                    // learned coarse correction (rr_mlp_init)
  double* mlp_scale = nullptr;    // device scalar ||P^T r|| of the learned correction
  struct PowerWork {              // buffers of the power-iteration smoother weight
    double *v = nullptr, *t = nullptr, *u = nullptr, *D = nullptr, *vin = nullptr;
    double *parts = nullptr, *nrm = nullptr;
  };
  PowerWork* pw = nullptr;
  int nblk = 0;                   // block smoother: blocks of <= 32 features
  int* boff = nullptr;            // [nblk+1] offsets into bperm
  int* bperm = nullptr;           // [F] internal features in block order
  double* bgram = nullptr;        // [nblk * 32 * 32] X_B^T X_B, row-major, zero-padded
  rr::DenseX* dense = nullptr;    // rr_setup_dense: X is dense (no sparse X)
  rr::DenseWork* dwork = nullptr;
  rr::Work w;                     // work set 0
  std::vector<rr::Work*> extra_sets;   // work sets 1, 2, ... for concurrent solves
  int npartials = 0;
  double* omega_tmp = nullptr;    // device scalar for the smoother weight
  double setup_ms = 0, kmeans_ms = 0, tune_ms = 0;
  rr::SellTuning tuning;
  std::vector<hipEvent_t> ev_pool;
  hipStream_t bstream = nullptr;    // the handle's own stream for batched solves
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

#define RR_HIP_VOID(call) (void)(call)

#define RR_TRY(call)                                                         \
  do {                                                                       \
    rr_status s_ = (call);                                                   \
    if (s_ != RR_OK) return s_;                                              \
  } while (0)

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// ---- sparse kernels (spmv.hip) ----------------------------------------------
rr_status build_chunk_plan(MergePlan& mp, const int* d_seg_ptr, int nseg, hipStream_t s);
rr_status build_cluster_rows(rr_handle* h, hipStream_t s);
void free_cluster_rows(ClusterRows& cr);
void launch_cluster_rows(const rr_handle* h, const double* yc, const double* rw, double* u, const int* done,
                         hipStream_t s);
void launch_row_scale(int N, const double* rw, const double* in, double* out, hipStream_t s);
rr_status gram_rows(const double* Xc, int fc, int FCp, int Np, double* K, hipStream_t s);
rr_status weighted_gram_from_labels(rr_handle* h, hipStream_t s);
rr_status leader_follower(rr_handle* h, double tol, int* fc, hipStream_t s);
void launch_cluster_rows32(const rr_handle* h, const double* yc, float* u, const int* done, hipStream_t s);
rr_status build_merge_plan(MergePlan& mp, const int* d_seg_end, const int* d_seg_ptr,
                           int nseg, int nnz, hipStream_t s);
void free_merge_plan(MergePlan& mp);
// u = X v (CSR).  done may be null.
// With `mid`, an event is recorded after the gather kernel of a sliced pass
// (before its segment reduction); elsewhere after the whole pass.
void launch_csr(const Sparse& X, const double* v, double* u, const int* done, hipStream_t s,
                const StageArgs* stage = nullptr, hipEvent_t mid = nullptr);
// up = X z + beta up (with row weights D: D X z + beta up), beta formed from
// pu as the PCG direction update takes it: X p of the new direction from X p
// of the previous one (0/1 X with the row-pass plan only: csr_pupd_ok).
bool csr_pupd_ok(const Sparse& X);
void launch_csr_pupd(const Sparse& X, const double* z, double* up, const int* done, hipStream_t s,
                     const PUpd& pu, hipEvent_t mid = nullptr);
// Column-segment reduction t_s = sum_e v[idx[e]] (* val[e]) with epilogue `mode`.
// Epilogues with a dot product leave block partials in e.partials; the
// return value is their count (0 for the other modes).
int launch_segsum(const MergePlan& mp, const int* seg_end, const int* idx, const double* val,
                  const double* v, int mode, const Epi& e, const int* done, hipStream_t s);
// X^T u with epilogue, using the CSC of X; returns the partial count.
int launch_csc(const Sparse& X, const double* u, int mode, const Epi& e, const int* done,
               hipStream_t s, hipEvent_t mid = nullptr);
rr_status build_csc(Sparse& X, hipStream_t s);
rr_status renumber_features(Sparse& X, int* fperm, int* finv, hipStream_t s);
// The operator's plans for 0/1 X: the row pass (lanes per row) and the sliced
// column pass (lane-stream target nnz / (CUs x 16 waves x 64 lanes x div),
// clamped to [8, 64]).  With autotune, lanes per row and the divisor are
// chosen among {1, 2, 4} by timing, once per device and shape bucket.
rr_status build_sell_plans(Sparse& X, hipStream_t s, int autotune, SellTuning* tuned);
void free_sell(SellPlan& sp);
int launch_sell(const SellPlan& sp, const double* v, int mode, const Epi& e, const int* done,
                hipStream_t s, const StageArgs* stage = nullptr, hipEvent_t mid = nullptr);
int sell_reduce_grid(const SellPlan& sp);
// Single-precision pass over v (float) with FP32 sums into `part` (float
// [sp.nout], the caller's); returns the count of dot partials left.
int launch_sell32(const SellPlan& sp, float* part, const float* v, int mode, const Epi32& e,
                  const int* done, hipStream_t s, const StageArgs* stage = nullptr);
// The gather kernel alone (partial sums only; no reduction, no epilogue).
void launch_sell_gather(const SellPlan& sp, const double* v, hipStream_t s, const int* done = nullptr);
// The column pass of X P for 0/1 X: segment s = cluster s holds the rows of
// every entry of X in a column of cluster s (rows ascending, repeated once
// per entry), so the pass's pieces add up to ((X P)^T u)_s / P_js.  rp/ci:
// X's CSR on the host, lab: the cluster of every feature.
rr_status build_xp_plan(SellPlan& xp, const std::vector<int>& rp, const std::vector<int>& ci,
                        const std::vector<int>& lab, int N, int FC, int num_cu, int div, hipStream_t s);
void launch_rows(const RowPlan& rp, const double* v, double* u, const double* scale, const int* done,
                 hipStream_t s, const StageArgs* stage = nullptr);
void launch_rows_pupd(const RowPlan& rp, const double* z, double* up, const double* scale, const int* done,
                      hipStream_t s, const PUpd& pu);
void launch_rows32(const RowPlan& rp, const float* v, float* u, const int* done, hipStream_t s,
                   const StageArgs* stage = nullptr);
void free_rows(RowPlan& rp);
rr_status build_batch_plan(BatchPlan& bp, const Sparse& X, hipStream_t s, int autotune);
void free_batch_plan(BatchPlan& bp);
void launch_batch_solve(const BatchProb* probs, const int* order, int nprob, int* queue, BatchOut* out,
                        int grid, hipStream_t s);
void launch_batch_gram(const BatchProb* probs, int nprob, const double* const* vin, int grid, hipStream_t s);
rr_status batch_scratch(BatchScratch* out);
rr_status lanczos_prototypes(rr_handle* h, int n_proto, int steps, uint64_t seed, double* V, double* ev,
                             hipStream_t s);
rr_status build_rows(RowPlan& out, const std::vector<int>& ptr, const std::vector<int>& col, int N, int F,
                     int num_cu, int L, hipStream_t s, const std::vector<double>* val = nullptr);
// More than kMaxParts block partials are first added into partials[0] by one
// block; returns the count the consumer should add.
int collapse_parts(double* partials, int n, const int* done, hipStream_t s);
rr_status validate_csr(const Sparse& X, hipStream_t s);

// ---- vector kernels (blas1.hip) ---------------------------------------------
enum PcgKind { PK_NONE = 0, PK_JACOBI = 1, PK_VCYCLE = 2, PK_ADDITIVE = 3, PK_LEARNED = 4,
               PK_ROUGHER = 5 };
int vec_grid(int F);   // blocks of the PCG vector kernels (<= kMaxParts)
void launch_pcg_init(int F, const double* b, double* x, double* r, double* p, double* z,
                     double* e1, const double* D, const double* xref, double omega, int kind,
                     double* parts_init, hipStream_t s);
void launch_finish_init(Scalars* sc, const double* parts_init, int n, double* history, int kind,
                        hipStream_t s);
void launch_pcg_update(int F, double* x, double* r, const double* p, const double* q,
                       double* z, double* e1, const double* D, const double* xref,
                       double omega, int kind, Scalars* sc, const double* parts_pq, int n_pq,
                       double* parts_upd, hipStream_t s);
// p = z + beta p; beta from rz partials (first: beta = 0); with `stage` the
// convergence check of the preceding update runs first
void launch_pupdate(int F, double* p, const double* z, Scalars* sc, const double* parts_rz,
                    int n_rz, int first, const StageArgs* stage, hipStream_t s);
void launch_stage_update(const StageArgs& st, hipStream_t s);
void launch_finish_true(Scalars* sc, const double* parts, int n, hipStream_t s);
void launch_fcg_dots(int F, const double* z, const FcgWindow& win, double* parts, Scalars* sc,
                     const StageArgs* stage, hipStream_t s);
void launch_fcg_dir(int F, const double* z, const double* r, double* p, const FcgWindow& win,
                    const double* dots, const double* paps, double* parts_pr, const Scalars* sc,
                    hipStream_t s);
void launch_fcg_update(int F, double* x, double* r, const double* p, const double* q, double* z,
                       double* e1, const double* D, const double* xref, double omega, int kind,
                       Scalars* sc, const double* parts_pq, int n_pq, const double* parts_pr,
                       double* paps, int slot, double* parts_upd, hipStream_t s);
void launch_prolong(int F, const int* labels, const double* cscale, const double* yc,
                    const double* e1, double* out, const double* r, const double* D,
                    double omega, int additive, const Scalars* sc, double* parts_rz,
                    hipStream_t s, const double* pw = nullptr);
void launch_fill(double* x, double v, long long n, hipStream_t s);
// ---- single-precision inner solves (mixed.hip) -------------------------------
void launch_cycle_in(int F, const double* r64, const double* colnorm, double lam, double omega,
                     const IrVectors& v, const int* done, hipStream_t s);
void launch_widen(int F, const float* z32, double* z, const int* done, hipStream_t s);
void launch_ir_init(int F, const double* r64, const double* colnorm, double lam, double omega,
                    int kind, const IrVectors& v, double* parts, hipStream_t s);
void launch_ir_update(int F, const IrVectors& v, double omega, int kind, Scalars* sc,
                      const double* parts_pq, int n_pq, double* parts_upd, hipStream_t s);
void launch_ir_pupdate(int F, float* p, const float* z, Scalars* sc, const double* parts_rz,
                       int n_rz, int first, const StageArgs* stage, hipStream_t s);
void launch_prolong32(int F, const int* labels, const double* cscale, const double* yc,
                      const float* e1, float* e2, const int* done, hipStream_t s);
void launch_ir_accumulate(int F, double* x, const float* d, hipStream_t s);
// dst[i] = src[idx[i]]
void launch_gather(double* dst, const double* src, const int* idx, int n, hipStream_t s);
void launch_copy(double* dst, const double* src, long long n, hipStream_t s);
void launch_copy_done(double* dst, const double* src, int n, const int* done, hipStream_t s);
void launch_colnorm_diag(int F, const double* colnorm, double lam, double* D, hipStream_t s);
void launch_jacobi_apply(int F, const double* r, const double* D, double* z, hipStream_t s);
void launch_omega_gersh(int F, const double* g, const double* colnorm, double lam,
                        double* out, double* partials, unsigned* ticket, hipStream_t s);
void launch_gemv(int n, const double* A, const double* x, double* y, const int* done,
                 hipStream_t s);

// ---- learned coarse correction (mlp.hip) -------------------------------------
void free_mlp(Mlp& n);
rr_status mlp_alloc(Mlp& n, int in, int hid, int out, int max_batch);
rr_status mlp_set(Mlp& n, const float* host, hipStream_t s);
void mlp_load_inputs(Mlp& n, const float* X, const int* rows, int Bn, hipStream_t s);
void mlp_forward(Mlp& n, int Bn, hipStream_t s);
void mlp_set_dout(Mlp& n, const float* dY, int Bn, hipStream_t s);
void mlp_loss_grad(Mlp& n, const float* T, const int* rows, int Bn, hipStream_t s);
void mlp_backward(Mlp& n, int Bn, hipStream_t s);
void mlp_adam(Mlp& n, float lr, hipStream_t s);
void launch_learned_in(int FC, const double* c, double lam, uint16_t* xb, double* scale,
                       const int* done, hipStream_t s);
void launch_learned_out(int FC, const float* y, const double* scale, const double* K, double lam, double* yc,
                        const int* done, hipStream_t s);
void launch_make_pairs(int FC, int npairs, const double* S, const double* Ainv_rc, const double* K, double lam,
                       float* inputs, float* targets, hipStream_t s);

// ---- coarse level (coarse.hip) ---------------------------------------------
rr_status coarse_factor(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s);
constexpr int kMaxJacobiSweeps = 40;
rr_status coarse_eigen(rr_handle* h, int* sweeps, hipStream_t s);
rr_status coarse_from_eigen(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s);
void launch_noise_rhs_in(int N, const double* y, const double* xi1, double a, double* v, hipStream_t s);
void launch_axpy_out(int F, double* b, const double* xi2, double c, hipStream_t s);

// ---- clustering (kmeans.hip) -----------------------------------------------
uint64_t splitmix64_next(uint64_t& state);   // SplitMix64 (Steele, Lea & Flood)
rr_status run_kmeans(rr_handle* h, int k, uint64_t seed, int max_iter, hipStream_t s);
rr_status set_labels(rr_handle* h, const int* labels_in, int nlab, hipStream_t s);
rr_status build_coarse_gram(rr_handle* h, hipStream_t s);
rr_status check_coarse_size(int fc);   // RR_ERR_UNSUPPORTED above 18,944 clusters (0/1 X)
rr_status build_coarse_gram_valued(rr_handle* h, hipStream_t s);   // (api.hip)
// c = P^T v over the restriction plan mp (either interpolation)  (api.hip)
void launch_restrict(const rr_handle* h, const MergePlan& mp, const double* v, double* out,
                     const int* done, hipStream_t s);
// the restriction from cluster-ordered v and the coarse GEMV yc = Ainv c in two
// kernels, the restriction's finishing step folded into the GEMV (c then holds
// the short clusters' entries only); usable when restrict_gemv_fusable
bool restrict_gemv_fusable(const MergePlan& mp, int n);
void launch_restrict_gemv(const MergePlan& mp, const double* v_sorted, const double* val, const double* scale,
                          double* c, int n, const double* Ainv, double* yc, const int* done, hipStream_t s);
// The restriction of r - A e1 and the coarse GEMV from the row pass's u = X e1
// (V(1,1), 0/1 X, square-root-average P): launch_sell_gather of the X P plan
// xp into xpart first; then c_s = P_js (sum_{j in s} (r_j - lam e1_j) - the
// cluster's xp pieces) and yc = Ainv c, in two kernels.  mp: the plan of
// build_xp_restrict (with this work set's cpart), perm: the cluster order;
// usable when restrict_gemv_fusable(mp, n).
void launch_restrict_gemv_xp(const MergePlan& mp, const int* perm, const double* r, const double* e1, double lam,
                             const double* scale, const SellPlan& xp, const double* xpart, double* c, int n,
                             const double* Ainv, double* yc, const int* done, hipStream_t s);
// Wave items of that restriction (setup only): the restriction plan's items
// over the clusters (offsets d_coff into the cluster order of F features),
// except that a cluster with more than 128 X P pieces (or more than 1024
// members) is finished from chunk sums, with extra items that sum its pieces
// 512 at a time.
rr_status build_xp_restrict(MergePlan& mp, const SellPlan& xp, const int* d_coff, int FC, int F, hipStream_t s);
// the same from v stored in cluster order (v[k] belongs to feature perm[k])
void launch_restrict_sorted(const rr_handle* h, const MergePlan& mp, const double* v, double* out,
                            const int* done, hipStream_t s);
// least-squares interpolation weights from prototypes  (interp.hip)
rr_status set_interpolation(rr_handle* h, const double* V, int nproto, double beta, const int* rep,
                            double* p_out, hipStream_t s);
void free_interpolation(rr_handle* h);

// ---- CG rougher (blas1.hip) --------------------------------------------------------
// With D non-null the steps are Jacobi-preconditioned (z = D^-1 res).
// Stage check of the preceding update, then p = z and <r, z> partials.
void launch_rg_start(int F, const double* r, const double* D, double* p, double* rr_parts,
                     Scalars* sc, const StageArgs* stage, hipStream_t s);
// alpha = rz / pq; e = (first ? 0 : e) + alpha p; res = (first ? r : res) - alpha q;
// <res, z> partials
void launch_rg_step(int F, int first, const double* r, const double* D, double* e, double* res,
                    const double* p, const double* q, const double* rr, int n_rr, const double* pq,
                    int n_pq, double* rr_out, const Scalars* sc, hipStream_t s);
// p = z + (rz_new / rz_old) p
void launch_rg_dir(int F, const double* res, const double* D, double* p, const double* rr_new,
                   int n_new, const double* rr_old, int n_old, const Scalars* sc, hipStream_t s);

// ---- block smoother (block.hip) ------------------------------------------------
constexpr int kSmoothBlock = 32;
rr_status build_smoother_blocks(rr_handle* h, hipStream_t s);
rr_status block_factor(rr_handle* h, double lam, LambdaSlot& slot, hipStream_t s);
// out = base + omega D_B^-1 rho + P yc (base, yc optional), over internal
// features; with parts: one <r, out> partial per workgroup, count returned.
int launch_block_smooth(const rr_handle* h, const double* Dinv, double omega, const double* rho,
                        const double* base, const double* yc, const double* r, double* out,
                        double* parts, const int* done, hipStream_t s);

// ---- dense X (dense.hip) -------------------------------------------------------
rr_status dense_setup(rr_handle* h, const rr_dense* X, const rr_setup_opts* o, hipStream_t s);
void dense_free(rr_handle* h);
rr_status dense_coarse_gram(rr_handle* h, hipStream_t s);
// t = A v + 0 (EPI_APPLY with lam) for one F-vector in FP64 (power iteration)
rr_status dense_apply_one(rr_handle* h, const double* v, double lam, double* t, hipStream_t s);
rr_status dense_solve_block(rr_handle* h, double lam, int m, const double* rhs, int64_t ld_rhs,
                            double* w, int64_t ld_w, const rr_solve_opts* o, rr_solve_info* info,
                            hipStream_t s);
rr_status dense_apply_block(rr_handle* h, double lam, int m, const double* v, int64_t ldv,
                            double* q, int64_t ldq, int precision, hipStream_t s);
rr_status dense_kmeans(rr_handle* h, int k, uint64_t seed, int max_iter, hipStream_t s);
// the cached coarse factor and smoother weight for lambda (api.hip)
rr_status get_slot_dense(rr_handle* h, double lam, LambdaSlot** out, hipStream_t s);

}  // namespace rr
