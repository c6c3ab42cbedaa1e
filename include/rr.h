/*
 * rr.h -- C ABI of the MI355X two-level preconditioned CG solver for the
 * regularized normal equations (X^T X + lambda I) w = X^T y.
 *
 * Method (Tavernier, Simm, Meerbergen, Moreau, "Two-level preconditioning
 * for Ridge Regression", arXiv 1806.05826):
 *   - the system and the ridge solution: introduction and the ridge
 *     regression subsection (the paper's beta is lambda here);
 *   - the two-level preconditioner: the two-level iteration subsection
 *     (Galerkin coarse level, pre/post smoothing), with the adjusted
 *     square-root average prolongation P (P(j,s) = 1/sqrt(n_s)) and the
 *     Galerkin coarse matrix A_c = P^T A P = X_c^T X_c + lambda I of the
 *     data-matrices subsection;
 *   - the aggregation: K-means++ over the feature columns (clustering
 *     section, K-means++ subsection), Euclidean distance;
 *   - the coarse solve: Cholesky (experiments section);
 *   - the Krylov iteration: PCG from x0 = 0, r0 = b, stopped on the
 *     relative residual (initialisation of the flexible CG algorithm; the
 *     residual plotted in the experiments).
 * Beside these: flexible CG with the CG pre-smoother of the experiments
 * (TLFCG), leader-follower clustering (clustering section), least-squares
 * interpolation of prototype vectors (rr_set_interpolation), the
 * eigendecomposition of the coarse Gram matrix for many lambda and the
 * noise-injection right-hand side of Bayesian regression (rr_coarse_eigen,
 * rr_noise_rhs), the weighted operator X^T D X + beta I of Newton steps
 * (rr_set_row_weights), and a learned coarse correction (rr_mlp_*).
 *
 * Conventions for every entry point:
 *   - Every call returns rr_status; RR_OK (0) on success.  On any other
 *     status rr_last_error() returns a message for the calling thread.
 *     No C++ exception or abort crosses the ABI.
 *   - Pointers documented "device" are HIP device pointers of the current
 *     device; "host" pointers are ordinary host memory.  The library never
 *     takes ownership of caller memory.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Calls are ordered on that stream; calls that return host-visible
 *     results (info structs, rr_smoother_weight) synchronize it.
 *   - Vectors are FP64, contiguous.  F-vectors are indexed by feature in
 *     the caller's column order; N-vectors by sample.
 *   - A handle is not thread-safe: one call at a time per handle.  Several
 *     handles may be used concurrently on different streams.
 *   - Device memory for a handle is allocated by rr_setup (rr_setup_dense)
 *     and released by rr_destroy.  Some buffers are allocated on first use
 *     and kept until rr_destroy: further work sets of rr_solve_batched, the
 *     FCG direction ring, the FP32 vectors of single-precision inner
 *     solves, the power-iteration buffers of the smoother weight, an extra
 *     per-lambda factor slot while every cached one is in use by a running
 *     solve, and the weights of rr_set_row_weights and
 *     rr_set_interpolation.  Repeating a solve of a kind the handle has
 *     already run allocates nothing; the set-up calls (rr_set_row_weights,
 *     rr_set_interpolation, rr_collect_pairs, rr_mlp_init, rr_mlp_train)
 *     may also allocate and free temporaries.
 */
#ifndef RR_H
#define RR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RR_OK = 0,
  RR_ERR_INVALID_ARG = 1,   /* bad size, pointer, option or input matrix   */
  RR_ERR_DEVICE = 2,        /* a HIP call failed                            */
  RR_ERR_WORKSPACE = 3,     /* the caller's workspace is too small          */
  RR_ERR_NOT_CONVERGED = 4, /* max_iter reached; w holds the last iterate   */
  RR_ERR_BREAKDOWN = 5,     /* <p,Ap> or <r,z> not positive / not finite    */
  RR_ERR_UNSUPPORTED = 6    /* valid request this build does not implement  */
} rr_status;

/* Preconditioner B used by rr_solve / rr_apply_precond (z = B r). */
typedef enum {
  RR_PRECOND_NONE = 0,     /* plain CG: z = r                                   */
  RR_PRECOND_JACOBI = 1,   /* DCG: z = D^-1 r, D = diag(A) = ||x_j||^2 + lambda  */
  RR_PRECOND_VCYCLE = 2,   /* two-level cycle, damped-Jacobi pre/post smoothing:
                              e1 = w D^-1 r; rho1 = r - A e1;
                              e2 = e1 + P A_c^-1 P^T rho1; rho2 = r - A e2;
                              z = e2 + w D^-1 rho2  (three operator applications
                              per PCG iteration, SPD for w rho(D^-1 A) < 2)      */
  RR_PRECOND_ADDITIVE = 3, /* z = w D^-1 r + P A_c^-1 P^T r                      */
  RR_PRECOND_LEARNED = 4,  /* the VCYCLE cycle with its coarse solve replaced by
                              the network: e2 = e1 + P yc, yc_s = ||r_c|| y_s /
                              (K_ss + lambda), y its output for [r_c / ||r_c||,
                              log lambda], r_c = P^T rho1, K = P^T X^T X P
                              (rr_mlp_init / rr_mlp_train); no coarse Cholesky
                              is applied; nonlinear, so flexible CG only; after
                              an iteration chunk that reduces ||r|| by less than
                              10 %, or a step whose <p,Ap> is not positive and
                              finite or whose <p,r> is not finite (a network
                              giving NaN or Inf), the solve continues from the
                              last good iterate with RR_PRECOND_VCYCLE and a
                              fresh flexible-CG history (info.fallback_iter)   */
  RR_PRECOND_ROUGHER = 5   /* the configuration of the paper's experiments
                              (TLFCG): rougher_steps iterations of plain CG on
                              A e = r from e = 0 as pre-smoother, then
                              z = e1 + P A_c^-1 P^T (r - A e1) with the CG
                              recurrence residual; no post-smoothing;
                              nonlinear, so flexible CG only                    */
} rr_precond;

typedef struct rr_handle rr_handle;
typedef void* rr_stream;

/* Sparse feature matrix X (N x F) in CSR form, 0-based. */
typedef struct {
  int64_t n_rows;          /* N >= 1                                           */
  int64_t n_cols;          /* F >= 1                                           */
  int64_t nnz;             /* >= 0, < 2^31                                     */
  const int32_t* row_ptr;  /* device int32[N+1], row_ptr[0] = 0, non-decreasing */
  const int32_t* col_idx;  /* device int32[nnz], strictly increasing per row    */
  const double* values;    /* device double[nnz], or NULL for a 0/1 (binary)
                              matrix: every stored entry is 1                  */
} rr_csr;

/* Dense feature matrix X (N x F), row-major FP32 (the dense case of the
 * data-matrices subsection: real-valued samples, every feature stored). */
typedef struct {
  int64_t n_rows;          /* N >= 1                                           */
  int64_t n_cols;          /* F >= 1                                           */
  int64_t ld;              /* >= F: elements between consecutive rows          */
  const float* values;     /* device float[N * ld], finite                     */
} rr_dense;

/* Option structs are versioned: struct_size must hold sizeof(the struct) as
 * the caller's copy of this header defines it.  The library reads that many
 * bytes; fields past them (a caller built against an older header) take
 * their defaults.  struct_size = 0 is rejected (RR_ERR_INVALID_ARG), so a
 * zero-initialised struct must still set it.  A NULL options pointer means
 * every default. */
typedef struct {
  uint32_t struct_size;    /* sizeof(rr_setup_opts)                             */
  int32_t n_clusters;      /* k >= 1: k-means++ clusters of the feature columns;
                              0: no coarse level (only NONE/JACOBI solves)      */
  int32_t kmeans_max_iter; /* Lloyd assignment passes; 0 -> 100                 */
  uint64_t seed;           /* SplitMix64 seed of the k-means++ draws            */
  const int32_t* labels_in;/* optional device int32[F]: use this aggregation
                              (labels in [0, n_labels_in)) instead of k-means;
                              empty labels are dropped and the rest renumbered
                              in increasing order                              */
  int32_t n_labels_in;
  int32_t lambda_slots;    /* coarse factors cached per handle; 0 -> 4          */
  int32_t autotune;        /* sparse X: 1 chooses each sliced pass's lane-stream
                              length among three candidates by timing them on
                              this device, cached per device and shape bucket
                              (log2 of N, F, nnz) for the life of the process,
                              and, for 0/1 X with F <= 8192, the persistent
                              batched solve's lanes per row (the default, half
                              and twice it, timed on one workgroup, cached the
                              same way);
                              dense X: 1 chooses the split of the column pass's
                              contraction (the workgroups it aims at, one of
                              128..2048) per operator precision, timed on a
                              256-column block, cached per device and shape
                              bucket (log2 of the padded N, F)                 */
  int32_t block_smoother;  /* sparse X with a coarse level: 1 also builds the
                              cluster-aligned smoother blocks (each cluster's
                              features in increasing index, cut into groups of
                              at most 32) and their Gram matrices X_B^T X_B,
                              for solves with smoother = RR_SMOOTHER_BLOCK     */
  int32_t coarse_eigen;    /* with a coarse level: 1 also forms K = Q diag(ev) Q^T
                              (parallel cyclic Jacobi, FP64) at setup; the
                              solves then take A_c(lambda)^-1 = Q diag(1/(ev +
                              lambda)) Q^T, one GEMM per new lambda instead of
                              a Cholesky factorization (the SVD coarse solver
                              of the Bayesian-regression experiments)          */
  double lf_tolerance;     /* 0/1 X: > 0 selects leader-follower clustering of
                              the feature columns instead of k-means (the
                              aggregation of the paper's experiments): in the
                              caller's feature order, a feature follows the
                              nearest earlier leader (ties: the earliest) if
                              its Euclidean distance is < lf_tolerance, else
                              it becomes the next leader; leaders are not
                              updated.  n_clusters is then ignored and
                              rr_get_centres returns the leaders in creation
                              order.  At most 18,944 clusters (the exact
                              integer coarse Gram matrix keeps a histogram of
                              F_C counts per workgroup in LDS)              */
  /* Buffers of later solves, reserved here so that those solves allocate
   * nothing (see "Device memory" below).  Solves that need more than was
   * reserved allocate it then, or fail with RR_ERR_WORKSPACE on a handle
   * set up on a caller workspace. */
  int32_t reserve_fcg_m;   /* flexible-CG directions (fcg_m of later solves)   */
  int32_t reserve_sets;    /* work sets beyond the handle's own, for
                              rr_solve_batched with the handle several times */
  int32_t reserve_f32;     /* 1: the vectors of RR_PREC_F32_IR solves (0/1 X) */
  int32_t reserved0;
} rr_setup_opts;

/*
 * rr_setup: copy X (device CSR) into library-owned storage, build its CSC
 * transpose, the column norms ||x_j||^2 and the Gershgorin row sums of
 * X^T X, then the aggregation (k-means++ over the columns, exact integer
 * arithmetic for binary X) and the lambda-independent coarse Gram matrix
 * K = P^T X^T X P.  X's arrays are only read during the call.  For non-binary
 * X the k-means aggregation is not implemented (RR_ERR_UNSUPPORTED): pass
 * labels_in; K is then formed one coarse column at a time, K e_c =
 * P^T X^T X (P e_c), in FP64 (F_C operator applications at setup).
 * Errors: RR_ERR_INVALID_ARG for an invalid matrix (bad row_ptr, column index
 * out of range or not increasing) or options; RR_ERR_DEVICE on HIP failure.
 * On success *out receives a handle to release with rr_destroy.
 */
rr_status rr_setup(const rr_csr* X, const rr_setup_opts* opts, rr_stream stream,
                   rr_handle** out);

/* Release a handle and its device memory (NULL is a no-op). */
rr_status rr_destroy(rr_handle* h);

/*
 * Device memory.  A handle takes its device memory, at setup and whenever a
 * later call needs more (for instance a larger flexible-CG ring than was
 * reserved), from one of three sources, fixed when it is set up:
 *   - a caller workspace (rr_setup_ws): the handle lives inside that buffer,
 *     which the caller allocates (for instance as a PyTorch tensor), keeps
 *     alive and unmodified until rr_destroy, and frees afterwards.  The
 *     library never frees it; a request that does not fit fails with
 *     RR_ERR_WORKSPACE;
 *   - the caller's allocator installed with rr_set_allocator when the handle
 *     was set up (the Python binding installs PyTorch's caching allocator):
 *     alloc(bytes, device, ctx) returns device memory or NULL, free(ptr,
 *     device, ctx) takes it back; the library frees only after synchronising
 *     the device, so no queued work still uses the block;
 *   - otherwise hipMalloc / hipFree.
 * Once a handle's solve buffers are reserved (rr_setup_opts.reserve_*),
 * rr_solve, rr_solve_batched (with distinct handles or reserved work sets,
 * lambdas whose factors fit the lambda_slots) and the operator and
 * preconditioner calls allocate no device memory.  The persistent batched
 * solve keeps per-device descriptor buffers, taken from the allocator current
 * at their first use and grown when a larger batch arrives.
 */
typedef void* (*rr_alloc_fn)(size_t bytes, int32_t device, void* ctx);
typedef void (*rr_free_fn)(void* ptr, int32_t device, void* ctx);
/* Install (both functions) or remove (both NULL) the caller's allocator for
 * handles set up from now on; existing handles keep their source. */
rr_status rr_set_allocator(rr_alloc_fn alloc, rr_free_fn free_fn, void* ctx);

/* *bytes = the workspace rr_setup_ws needs for this X and these options.
 * Computed exactly by running the setup once (with hipMalloc memory that is
 * released before returning): setup is deterministic, so an identical
 * rr_setup_ws call makes the same requests.  Costs one setup. */
rr_status rr_setup_workspace_size(const rr_csr* X, const rr_setup_opts* opts, rr_stream stream,
                                  size_t* bytes);

/* rr_setup with every device allocation of the handle carved out of the
 * caller's workspace (device memory, 256-byte aligned, ws_bytes bytes; too
 * small: RR_ERR_WORKSPACE).  The workspace must outlive the handle. */
rr_status rr_setup_ws(const rr_csr* X, const rr_setup_opts* opts, void* workspace, size_t ws_bytes,
                      rr_stream stream, rr_handle** out);

typedef struct {
  int64_t n_rows, n_cols, nnz;
  int32_t n_coarse;        /* F_C (clusters left after dropping empty ones)    */
  int32_t n_centres;       /* centres chosen by the seeding (fewer than k when
                              every feature coincides with a chosen centre)    */
  int32_t kmeans_iters;    /* Lloyd assignment passes run                      */
  int32_t binary;          /* 1 when X was given without values               */
  double setup_ms;         /* wall time of rr_setup                            */
  double kmeans_ms;        /* of which clustering                              */
  double plan_ms;          /* of which building (and tuning) the pass plans    */
  int32_t tuned_rows_div;  /* lanes per row of the row pass (1, 2, 4, 8 or 16)  */
  int32_t tuned_cols_div;  /* lane-stream divisor of the sliced column pass    */
  int32_t tune_cached;     /* 1: autotune reused an earlier measurement        */
  int32_t dense;           /* 1 for a handle made by rr_setup_dense (nnz =
                              n_rows * n_cols)                                 */
  int32_t dense_split[3];  /* dense X: workgroups the column pass's split
                              contraction aims at, for the FP64, BF16 and FP32
                              operators (tuned when autotune = 1)              */
  int32_t dense_split_cached; /* 1: those came from an earlier measurement     */
  int32_t eigen_sweeps;    /* coarse_eigen: Jacobi sweeps run (0: not formed)  */
} rr_setup_info;

/* Host-side facts about a handle. */
rr_status rr_get_setup_info(const rr_handle* h, rr_setup_info* info);

/* Copy the final labels (device int32[F], values in [0, F_C)). */
rr_status rr_get_labels(const rr_handle* h, int32_t* labels, rr_stream stream);

/* Copy the seeding centres in draw order (device int32[n_centres]). */
rr_status rr_get_centres(const rr_handle* h, int32_t* centres, rr_stream stream);

/* Arithmetic of rr_solve. */
typedef enum {
  RR_PREC_F64 = 0,         /* FP64 vectors, sums and scalars throughout          */
  RR_PREC_F32_IR = 1,      /* iterative refinement: r = b - A x and x in FP64;
                              each correction A d = r by PCG with FP32 vectors
                              and FP32 operator sums, FP64 scalars and FP64
                              coarse solve (0/1 X; none / Jacobi / V(1,1)).
                              Dense X (rr_solve_block): corrections with the
                              FP32-operand operator (FP32 matrix-core sums, U
                              in FP32) and FP64 vectors; inner_tol default 1e-5 */
  RR_PREC_BF16_IR = 2,     /* dense X (rr_solve_block): iterative refinement
                              whose corrections run PCG with a BF16-operand
                              operator (X and the input block rounded to BF16,
                              FP32 matrix-core sums, U = X V rounded to BF16),
                              FP64 vectors, scalars and coarse solve; the
                              residual b - A x uses the FP64 operator           */
  RR_PREC_F32_CYCLE = 3    /* 0/1 X, V(1,1), flexible CG: the Krylov space, its
                              operator q = A p, x, r and every scalar stay FP64
                              (so the solve reaches the FP64 tolerance without
                              restarts); the preconditioner's cycle runs in FP32
                              (r rounded, its two operator applications and
                              smoothing in FP32, the coarse solve in FP64) and
                              z is widened back.  Flexible CG absorbs the
                              cycle's rounding; reserve_f32 at setup reserves
                              its vectors                                       */
} rr_precision;

/* Smoother of the two-level cycle: S = omega D^-1 with D the diagonal of A
 * (point) or its cluster-aligned block diagonal D_B (blocks of <= 32
 * features inside one cluster, solved exactly).  The block form's automatic
 * weight is 1 / (1.1 rho), rho the norm ratio after 30 power steps
 * v <- D_B^-1 A v / ||.|| from the start vector of rr_smoother_weight. */
typedef enum {
  RR_SMOOTHER_POINT = 0,
  RR_SMOOTHER_BLOCK = 1
} rr_smoother;

/* Krylov method of rr_solve. */
typedef enum {
  RR_KRYLOV_PCG = 0,       /* preconditioned CG (needs a fixed SPD preconditioner) */
  RR_KRYLOV_FCG = 1        /* flexible CG with truncation fcg_m (the paper's
                              flexible-CG algorithm, Notay's FCG)                */
} rr_krylov;

typedef struct {
  uint32_t struct_size;    /* sizeof(rr_solve_opts)                              */
  int32_t reserved0;
  double tol;              /* stop when ||r_k|| <= tol ||b||; 0 -> 1e-10        */
  int32_t max_iter;        /* 0 -> 10000                                        */
  int32_t fixed_iters;     /* > 0: run exactly this many iterations              */
  int32_t precond;         /* rr_precond; VCYCLE/ADDITIVE need a coarse level    */
  int32_t rhs_is_b;        /* 0: rhs is y (device double[N]), b = X^T y;
                              1: rhs is b (device double[F])                     */
  double omega;            /* smoother weight w; 0 -> 1/rho_hat with rho_hat the
                              Gershgorin bound max_j (X^T X 1 + lambda)_j / D_j
                              (X >= 0), else a power-iteration estimate x 1.1   */
  const double* x_ref;     /* optional device double[F]: also stop as soon as
                              ||x_k - x_ref|| <= err_tol ||x_ref||               */
  double err_tol;
  double* residual_history;/* optional device double[limit+1]: ||r_k||/||b||    */
  int32_t chunk;           /* iterations queued between host checks; 0 -> 8      */
  int32_t profile;         /* 1: time every operator pass with HIP events; 2: also
                              time 20 back-to-back launches of each sliced gather
                              kernel on the final vectors; 3: the same with the
                              column pass's reduction in the second loop       */
  int32_t krylov;          /* rr_krylov: PCG (default) or flexible CG           */
  int32_t fcg_m;           /* flexible CG: directions kept, 1..16; 0 -> 1.
                              Direction i is orthogonalized against the
                              m_i = max(1, i mod (m+1)) previous ones (the
                              truncation of the paper's flexible-CG algorithm)  */
  int32_t precision;       /* rr_precision: FP64 (default) or FP32 inner solves
                              with FP64 iterative refinement                     */
  int32_t graph;           /* 1: PCG iterations are captured once per chunk
                              signature into a HIP graph and replayed (the
                              chunk's launches do not change between chunks);
                              ignored with profile, flexible CG and refinement  */
  double inner_tol;        /* refinement: relative residual of each inner solve;
                              0 -> 1e-4.  tol then bounds the FP64 residual
                              ||b - A x|| / ||b||, max_iter the inner iterations
                              of each step (at most 40 steps)                    */
  int32_t smoother;        /* rr_smoother of the two-level forms (V(1,1),
                              additive, learned): point Jacobi (default) or the
                              block smoother of a handle set up with
                              block_smoother = 1 (FP64 solves)                   */
  int32_t rougher_steps;   /* RR_PRECOND_ROUGHER: CG steps, 0 -> 2 (the paper's
                              choice), at most 16                                */
  int32_t rougher_jacobi;  /* RR_PRECOND_ROUGHER: 1 preconditions the rougher's
                              CG steps with the Jacobi diagonal (a variant; the
                              paper's rougher is plain CG)                       */
  int32_t persistent;      /* rr_solve_batched: 1 solves every problem in one
                              persistent kernel launch (replayed from a HIP
                              graph when graph = 1): a workgroup runs a whole
                              PCG solve, problems taken longest first.  2
                              (hybrid): the same launch, but a problem leaves
                              it after cap_i = hybrid_iters x (sum of costs
                              / CUs) / cost_i iterations (cost = nnz + N + F;
                              at least 16) and its PCG recurrence continues,
                              from the same x, r, p and <r,z>, with the
                              stream kernels of rr_solve_batched; the caps
                              depend on the sizes only, so results are
                              reproducible.  0/1 X
                              with at most 8192 features, FP64 PCG, V(1,1)
                              (n_coarse <= 5120) or Jacobi, point smoother,
                              no row weights or least-squares interpolation  */
  int32_t hybrid_iters;    /* persistent = 2: iterations of the cap formula; 0 -> 512 */
} rr_solve_opts;

typedef struct {
  int32_t status;          /* RR_OK / RR_ERR_NOT_CONVERGED / RR_ERR_BREAKDOWN    */
  int32_t iters;           /* PCG iterations (x updates)                         */
  int32_t op_applies;      /* operator applications, b = X^T y and the exit
                              residual excluded                                  */
  int32_t ir_steps;        /* refinement steps (RR_PREC_F32_IR), else 0         */
  double relres;           /* recursive ||r_k|| / ||b|| (refinement: the FP64
                              residual ||b - A x|| / ||b||)                      */
  double true_relres;      /* ||b - A x_k|| / ||b||, recomputed at exit          */
  double err;              /* ||x_k - x_ref|| / ||x_ref|| when x_ref is given    */
  double omega;            /* smoother weight used                               */
  double ms;               /* wall time of the call (persistent batched solves:
                              the problem's own time on its workgroup)          */
  double coarse_ms;        /* of which the per-lambda coarse factorization       */
  double csr_avg_ms;       /* profile: mean time of a row pass u = X v           */
  double csc_avg_ms;       /* profile: mean time of a column pass t = X^T u with
                              its epilogue                                       */
  int32_t csr_launches, csc_launches;
  double csr_gather_avg_ms;/* profile 1: of csr_avg_ms, the sliced gather kernel
                              (0/1 X; the whole pass for valued X); profile 2
                              and 3: its back-to-back launch time                */
  double csc_gather_avg_ms;/* profile 1, 2: the same for the column gather;
                              profile 3: the back-to-back time of the column
                              gather with its reduction and epilogue            */
  int32_t fallback_iter;   /* RR_PRECOND_LEARNED: iteration at which the solve
                              fell back to the algebraic cycle, else -1          */
  int32_t pad_;
} rr_solve_info;

/*
 * rr_solve: PCG on (X^T X + lambda I) w = b from w = 0 (or the fixed-
 * iteration / error-target variants above).  lambda must be finite and > 0.
 * `rhs` and `w` are device FP64 buffers owned by the caller; w receives the
 * last iterate also on RR_ERR_NOT_CONVERGED / RR_ERR_BREAKDOWN.  The call
 * blocks until *info (host) is valid.  The lambda-dependent coarse factor is
 * computed on first use of a lambda and cached in the handle.
 */
rr_status rr_solve(rr_handle* h, double lambda, const double* rhs, double* w,
                   const rr_solve_opts* opts, rr_solve_info* info, rr_stream stream);

/*
 * rr_solve_batched: nprob independent solves (the paper solves one system
 * per lambda, each with the two-level preconditioner of its own handle; its
 * amortization argument is that X, the clustering and K serve many solves).
 * Problem i solves (X_i^T X_i + lambdas[i] I) w = b_i on handles[i] with
 * rhs[i], w[i] as in rr_solve.  Host arrays: handles, lambdas, rhs, w (device
 * pointers), info[nprob] (may be NULL).  One options struct serves every
 * problem; x_ref and residual_history must be NULL (per-problem buffers) and
 * profile is ignored.  Problems run concurrently, each in a work set of its
 * handle (vectors, partial sums and a stream of its own; the k-th problem on
 * a handle uses the handle's k-th set, created on first use), with their
 * iteration chunks queued round-robin; beyond 8 problems per handle the rest
 * run in later waves.  Cached coarse factors in use are never evicted (the
 * cache grows instead).  Every problem's result is bitwise the result of
 * rr_solve with the same arguments.  The call
 * orders after prior work on `stream`, later work on `stream` orders after
 * it, and it blocks until info is valid.  Returns RR_OK when every problem
 * succeeded, else the first failing status (info[i].status per problem).
 * Errors: RR_ERR_INVALID_ARG for nprob < 0, null arrays or handles, or
 * per-problem buffers in opts.
 */
rr_status rr_solve_batched(int32_t nprob, rr_handle* const* handles, const double* lambdas,
                           const double* const* rhs, double* const* w, const rr_solve_opts* opts,
                           rr_solve_info* info, rr_stream stream);

/*
 * rr_solve_batched_noalloc: rr_solve_batched with persistent = 1 for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  It allocates nothing:
 * the problems' descriptors, launch order, records and queue counter live in
 * a static device array of the library (about 570 KB per GPU, held until the
 * process ends), so a call takes at most 2048 problems (more:
 * RR_ERR_INVALID_ARG).  Every handle must already hold what its problems
 * need: a handle listed k + 1 times needs k reserved work sets
 * (rr_setup_opts.reserve_sets) and, for V(1,1), no more distinct lambdas
 * than its lambda_slots (else RR_ERR_WORKSPACE).  The same restrictions as
 * the persistent solve apply (0/1 X, at most 8192 features, FP64 PCG, V(1,1)
 * or Jacobi).  The launch is never replayed from a graph (graph is ignored).
 * All calls on one GPU share its array: calls that overlap on one GPU race,
 * so a caller serialises them (the call returns only after its launch has
 * finished).
 */
rr_status rr_solve_batched_noalloc(int32_t nprob, rr_handle* const* handles, const double* lambdas,
                                   const double* const* rhs, double* const* w,
                                   const rr_solve_opts* opts, rr_solve_info* info, rr_stream stream);

/* Av = (X^T X + lambda I) v, v and Av device double[F] (lambda >= 0). */
rr_status rr_apply_operator(rr_handle* h, double lambda, const double* v, double* Av,
                            rr_stream stream);

/* b = X^T y, y device double[N], b device double[F] (row weights do not
 * apply). */
rr_status rr_apply_rhs(rr_handle* h, const double* y, double* b, rr_stream stream);

/* z = B r for the preconditioner `precond` (rr_precond) at this lambda;
 * omega = 0 selects the automatic weight.  r, z device double[F]. */
rr_status rr_apply_precond(rr_handle* h, double lambda, int32_t precond, double omega,
                           const double* r, double* z, rr_stream stream);

/* K = P^T X^T X P, device double[F_C * F_C] row-major (lambda-independent). */
rr_status rr_coarse_gram(rr_handle* h, double* K, rr_stream stream);

/* The Cholesky factor L (lower, row-major, zeros above the diagonal) of
 * A_c = K + lambda P^T P (P^T P = I for the adjusted square-root average,
 * diagonal under rr_set_interpolation) and A_c^-1, device double[F_C * F_C] each; either may be
 * NULL.  Errors: RR_ERR_BREAKDOWN if A_c is not numerically positive definite.
 * A handle set up with coarse_eigen forms A_c^-1 from the eigendecomposition
 * and no L: it returns RR_ERR_UNSUPPORTED when L is requested. */
rr_status rr_coarse_factor(rr_handle* h, double lambda, double* L, double* Ac_inv,
                           rr_stream stream);

/* The eigendecomposition K = Q diag(ev) Q^T formed with coarse_eigen: Q
 * device double[F_C * F_C] row-major (column k is the k-th eigenvector), ev
 * device double[F_C] (unsorted); either may be NULL.  RR_ERR_INVALID_ARG if
 * the handle was set up without coarse_eigen. */
rr_status rr_coarse_eigen(rr_handle* h, double* Q, double* ev, rr_stream stream);

/* The right-hand side of one noise-injection sample (the Bayesian
 * regression subsection, eq. ni_xtx): b = X^T (y + e1) + e2 / tau with
 * e1 = xi1 / sqrt(tau) ~ N(0, I_N / tau) and e2 = sqrt(lambda) xi2 ~ N(0,
 * lambda I_F), from the caller's standard-normal draws xi1 (device
 * double[N]) and xi2 (device double[F]).  The sample w solves
 * (X^T X + (lambda / tau) I) w = b: rr_solve with rhs_is_b at lambda / tau.
 * tau > 0 and lambda > 0, finite. */
rr_status rr_noise_rhs(rr_handle* h, double tau, double lambda, const double* y, const double* xi1,
                       const double* xi2, double* b, rr_stream stream);

/* Row weights d (device double[N], finite, >= 0; NULL clears them): from
 * here on the handle's operator is X^T D X + lambda I, D = diag(d), the
 * Hessian form of Newton steps for logistic regression and L2-loss SVMs
 * (the subsection on optimization by the Newton method).  The row pass
 * scales its output by d in the reduction's epilogue; solves from y form
 * b = X^T D y (rr_apply_rhs stays the plain X^T y, as a Newton gradient
 * needs).  The call rebuilds what depends on the
 * operator: the Jacobi diagonal sum_i d_i x_ij + lambda, the Gershgorin sums
 * X^T D X 1, the coarse matrix P^T X^T D X P (from the label table and one
 * FP64 GEMM through an F_C x N scratch matrix kept by the handle) and,
 * with coarse_eigen, its eigendecomposition; cached per-lambda factors and
 * captured graphs are dropped.  The aggregation P is kept.  0/1 X only,
 * without block-smoother blocks; no solve may run on the handle meanwhile.
 * Not with single-precision inner solves or rr_noise_rhs (RR_ERR_UNSUPPORTED).
 * RR_ERR_INVALID_ARG for a negative or non-finite weight. */
rr_status rr_set_row_weights(rr_handle* h, const double* d, rr_stream stream);

/* u = X v, the plain product whatever the row weights: v device double[F]
 * (caller's feature order), u device double[N]. */
rr_status rr_apply_rows(rr_handle* h, const double* v, double* u, rr_stream stream);

/* Least-squares interpolation (the least-squares interpolation subsection):
 * replaces the adjusted square-root average P by the P whose row j holds one
 * weight p_j in column labels[j], the minimiser of
 * sum_k eta_k (v_k(j) - p_j v_k(r))^2, i.e.
 *   p_j = sum_k eta_k v_k(j) v_k(r) / sum_k eta_k v_k(r)^2,
 * where r is the coarse feature of j's cluster and
 * eta_k = <(X^T X + beta I) v_k, v_k> (computed here with the operator).
 *   V      device double[n_proto * F]: prototype k is V[k*F .. k*F+F-1], in
 *          the caller's feature order (for instance the leading principal
 *          components of X^T X); read during the call only.  NULL restores
 *          the adjusted square-root average.
 *   n_proto 1..64.  beta >= 0, finite.
 *   rep    device int32[F_C]: the coarse feature (caller's index) of each
 *          cluster, which must be a member of it; NULL takes each cluster's
 *          member of lowest index (the leader under leader-follower).
 *   p      device double[F] (caller's order) receiving the weights, or NULL.
 * A cluster whose coarse feature has sum_k eta_k v_k(r)^2 = 0 keeps p_j = 1.
 * The coarse Gram K = P^T X^T X P is rebuilt with one operator application
 * per cluster, and A_c = K + lambda diag(P^T P); cached per-lambda factors and
 * captured graphs are dropped; no solve may run on the handle meanwhile.
 * The V(1,1) cycle's second row pass then runs as a full pass.  Solves with
 * the block smoother, the learned coarse correction or single-precision inner
 * solves return RR_ERR_UNSUPPORTED while it is set, and so do handles with
 * row weights or coarse_eigen.  RR_ERR_INVALID_ARG for a coarse feature
 * outside its cluster or prototypes giving non-finite weights (the previous
 * interpolation then stays). */
rr_status rr_set_interpolation(rr_handle* h, const double* V, int32_t n_proto, double beta,
                               const int32_t* rep, double* p, rr_stream stream);

/*
 * rr_prototypes: prototype vectors for rr_set_interpolation, the n_proto
 * leading eigenvectors of X^T X (the least-squares interpolation subsection
 * names the principal components of the data and computes them with Arnoldi
 * iterations; X^T X is symmetric, so Arnoldi is Lanczos here).  `steps`
 * Lanczos steps (0 -> max(30, 3 n_proto); n_proto <= steps <= 512) from a
 * fixed start vector (SplitMix64(seed) entries in [0.5, 1.5) in the caller's
 * feature order, normalised), every new basis vector orthogonalised twice
 * against the whole basis; the Ritz pairs of the projected tridiagonal
 * matrix give V (device double[n_proto * F], prototype k at V[k*F ..], the
 * caller's feature order, unit norm, each sign fixed by its largest Lanczos
 * coefficient) and ev (host double[n_proto], descending Ritz values).  The
 * Lanczos basis, (steps + 1) * F doubles, is allocated for the call.  A
 * Krylov space that closes before n_proto directions (X of lower rank)
 * returns RR_ERR_INVALID_ARG.  0/1 or valued sparse X.
 */
rr_status rr_prototypes(rr_handle* h, int32_t n_proto, int32_t steps, uint64_t seed, double* V,
                        double* ev, rr_stream stream);

/* The automatic smoother weight for this lambda (host double).  X >= 0: the
 * Gershgorin weight 1 / max_j (X^T X 1 + lambda)_j / D_j.  X with negative
 * entries: 1 / (1.1 rho), rho the norm ratio after 30 power iterations with
 * D^-1/2 A D^-1/2 from a fixed start vector whose entries, in the caller's
 * feature order, are u + 0.5 for u the successive SplitMix64 outputs of seed
 * 0x5eed mapped to [0, 1) by their top 53 bits, normalised to unit length.
 * Runs on the null stream with work set 0's buffers. */
rr_status rr_smoother_weight(rr_handle* h, double lambda, double* omega);

/*
 * Dense X with many right-hand sides.
 *
 * rr_setup_dense: copy X (device FP32, row-major) into four library-owned
 * copies (FP32 and BF16, X and X^T, zero-padded to multiples of 128 rows and
 * columns: 12 bytes per entry), the column norms ||x_j||^2 and, for X >= 0,
 * the Gershgorin sums X^T X 1 (FP64); then the aggregation (labels_in, or
 * k-means++ over the columns in FP64 on the matrix cores when n_clusters > 0)
 * and K = P^T X^T X P (FP64 matrix cores).  The options of rr_setup apply
 * (autotune tunes the column pass's split contraction).  Errors: RR_ERR_INVALID_ARG for bad sizes, a
 * non-finite entry or bad options; RR_ERR_DEVICE on HIP failure.  The handle
 * takes rr_solve_block, rr_apply_operator_block, rr_get_setup_info,
 * rr_get_labels, rr_get_centres, rr_coarse_gram, rr_coarse_factor,
 * rr_smoother_weight and rr_destroy; the other calls return
 * RR_ERR_UNSUPPORTED for it.
 */
rr_status rr_setup_dense(const rr_dense* X, const rr_setup_opts* opts, rr_stream stream,
                         rr_handle** out);

/*
 * rr_solve_block: nrhs systems (X^T X + lambda I) w_c = b_c with one lambda,
 * solved together: one operator application multiplies the whole block
 * (matrix-core GEMMs), every column keeps its own CG scalars, stopping test
 * and iteration count, and a converged column stays fixed.
 *   rhs: device double, column c at rhs + c * ld_rhs; y_c (N entries,
 *        ld_rhs >= N) or, with opts->rhs_is_b, b_c (F entries, ld_rhs >= F).
 *   w:   device double, column c at w + c * ld_w (ld_w >= F), written.
 *   opts: tol, max_iter, fixed_iters, precond (none / Jacobi / V(1,1) /
 *        additive), rhs_is_b, omega, precision (RR_PREC_F64: FP64 operator;
 *        RR_PREC_BF16_IR / RR_PREC_F32_IR: refinement with BF16- / FP32-operand
 *        corrections, inner_tol relative to each step's residual, default
 *        1e-3 / 1e-5); other fields must be zero.
 *   info: NULL or host rr_solve_info[nrhs], one per column (iters = PCG
 *        iterations, summed over refinement steps).
 * 1 <= nrhs <= 4096.  Returns RR_ERR_NOT_CONVERGED / RR_ERR_BREAKDOWN if any
 * column did; synchronizes the stream.
 */
rr_status rr_solve_block(rr_handle* h, double lambda, int32_t nrhs, const double* rhs,
                         int64_t ld_rhs, double* w, int64_t ld_w, const rr_solve_opts* opts,
                         rr_solve_info* info, rr_stream stream);

/* q_c = (X^T X + lambda I) v_c for nrhs columns (device double, leading
 * dimensions ldv, ldq >= F) of a dense handle, with the FP64 operator
 * (precision RR_PREC_F64), the FP32-operand one (RR_PREC_F32_IR) or the
 * BF16-operand one (RR_PREC_BF16_IR).
 * lambda >= 0.  Stream-ordered. */
rr_status rr_apply_operator_block(rr_handle* h, double lambda, int32_t nrhs, const double* v,
                                  int64_t ldv, double* q, int64_t ldq, int32_t precision,
                                  rr_stream stream);

/* Message for the last non-OK status on this thread ("" if none). */
const char* rr_last_error(void);

/*
 * ---- Learned coarse correction --------------------------------------------
 * A three-layer perceptron: in = F_C + 1 inputs [r_c / ||r_c||, log lambda],
 * two ReLU layers of `hidden` units, F_C outputs; the products run on the
 * matrix cores in BF16 with FP32 accumulation, master weights and Adam state
 * are FP32.  Parameters are handled as one FP32 array, row-major, in the order
 * W1 [hidden, in], b1 [hidden], W2 [hidden, hidden], b2 [hidden],
 * W3 [F_C, hidden], b3 [F_C].  None of this is in the paper; its flexible CG
 * is what admits such a nonlinear preconditioner.
 */
typedef struct {
  uint32_t struct_size;    /* sizeof(rr_mlp_train_opts)                            */
  int32_t epochs;          /* passes over the pairs; 0 -> 20                       */
  int32_t batch;           /* mini-batch size, 1..1024; 0 -> 256                   */
  double lr;               /* Adam step size; 0 -> 1e-3                            */
  uint64_t seed;           /* SplitMix64 seed of the per-epoch shuffles            */
} rr_mlp_train_opts;

/* Create (or re-create) the network of a handle with a coarse level:
 * He-uniform weights (bound sqrt(6/fan_in), SplitMix64(seed) draws in
 * parameter order), zero biases, fresh Adam state.  hidden in 16..1024. */
rr_status rr_mlp_init(rr_handle* h, int32_t hidden, uint64_t seed);

/* Sizes: parameter count, inputs, outputs. */
rr_status rr_mlp_size(const rr_handle* h, int64_t* n_params, int32_t* n_in, int32_t* n_out);

/* Copy the FP32 parameters from / to the host (n_params floats); setting
 * also resets the Adam state. */
rr_status rr_mlp_set_weights(rr_handle* h, const float* host_params);
rr_status rr_mlp_get_weights(const rr_handle* h, float* host_params);

/* out[b, :] = network(in[b, :]) for b < batch (device FP32 arrays [batch, in]
 * and [batch, F_C]); any batch size. */
rr_status rr_mlp_forward(rr_handle* h, const float* in, int32_t batch, float* out,
                         rr_stream stream);

/* Gradient of sum_b <dout[b], network(in[b])> with respect to the parameters
 * (device FP32 grads[n_params]); batch 1..1024. */
rr_status rr_mlp_backward(rr_handle* h, const float* in, const float* dout, int32_t batch,
                          float* grads, rr_stream stream);

/* Adam on the loss (1 / 2B) sum_b ||network(in[b]) - target[b]||^2 over
 * shuffled mini-batches of the n pairs (device FP32 in [n, F_C + 1],
 * target [n, F_C]).  loss_history (host, may be NULL) receives the mean loss
 * of every epoch. */
rr_status rr_mlp_train(rr_handle* h, const float* in, const float* target, int64_t n,
                       const rr_mlp_train_opts* opts, float* loss_history, rr_stream stream);

/* Training pairs generated by the solver: for each lambdas[i] (host) a V(1,1)
 * PCG solve of (X^T X + lambda I) w = X^T y (device y[N]) records the coarse
 * residual r_c = P^T rho1 that its cycle hands to the coarse solve, after
 * every `every`-th iteration, up to pairs_per_solve of them; pair q gets input
 * [r_c/||r_c||, log lambda] and target D_c A_c(lambda)^-1 r_c / ||r_c||, the
 * algebraic coarse correction in units of the coarse Jacobi step (D_c =
 * diag(A_c) = diag(K) + lambda I), so that targets are of order one whatever
 * the scale of A_c (RR_PRECOND_LEARNED divides the output by D_c again).
 * inputs [n_solves * pairs_per_solve, F_C + 1] and targets [.., F_C] are
 * device FP32; *n_pairs receives the count written (solves that converge
 * early give fewer). */
rr_status rr_collect_pairs(rr_handle* h, const double* lambdas, int32_t n_solves,
                           int32_t pairs_per_solve, int32_t every, const double* y, float* inputs,
                           float* targets, int64_t* n_pairs, rr_stream stream);

/* The same pairs from the network's own solves: for each lambdas[i] the
 * flexible CG solve with RR_PRECOND_LEARNED (truncation 4) records the
 * coarse residuals its cycle hands to the network, so a second training
 * round sees the residual directions a solve the network steers produces
 * (the V(1,1) solves of rr_collect_pairs never do).  Needs a network
 * (rr_mlp_init); the solves fall back as RR_PRECOND_LEARNED does, and the
 * residuals after a fallback come from the algebraic cycle. */
rr_status rr_collect_pairs_learned(rr_handle* h, const double* lambdas, int32_t n_solves,
                                   int32_t pairs_per_solve, int32_t every, const double* y,
                                   float* inputs, float* targets, int64_t* n_pairs, rr_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* RR_H */
