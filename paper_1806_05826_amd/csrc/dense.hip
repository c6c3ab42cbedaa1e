// Dense X with a block of right-hand sides (the real-valued, fully stored
// case of the data-matrices subsection): the operator Q = X^T (X V) + lam V
// as two matrix-core GEMMs, and block PCG with the two-level preconditioner
// of the two-level-iteration subsection, one set of CG scalars per column.
//
// Precisions: FP64 (FP64 MFMA, X widened from its FP32 copy) and BF16
// operands with FP32 accumulation (the corrections of iterative refinement,
// whose residual b - A x uses the FP64 operator).  Vectors, CG scalars and
// the coarse solve are FP64 in both.
//
// Layout: X in four copies (rr_internal.h, DenseX).  A block of m vectors is
// column-major; F-blocks have leading dimension Fp, N-blocks Np.  Every
// dimension a GEMM touches is a multiple of its tile, so the GEMMs have no
// bounds checks; the host checks that before each launch.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rr_device.h"

namespace rr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

void dense_free_work(DenseWork& W);

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

size_t rup(size_t a, size_t b) { return (a + b - 1) / b * b; }

template <typename T>
rr_status zalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  RR_HIP(dmalloc((void**)p, n * sizeof(T)));
  RR_HIP(hipMemset(*p, 0, n * sizeof(T)));
  return RR_OK;
}

template <typename T>
void zfree(T*& p) {
  if (p) (void)dev_free((void*)p);
  p = nullptr;
}

// Round to nearest even, FP32 -> BF16 (NaN kept quiet).
__device__ inline uint16_t bf16_of(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
// BF16 of an FP64 value: through FP32, each step rounding to nearest even.
__device__ inline uint16_t bf16_of(double x) { return bf16_of((float)x); }

// ---- GEMM, BF16 operands, FP32 accumulation ---------------------------------
//
// C[M x Nc] = A[M x K] B[K x Nc]; A row-major (lda), B column-major (ldb),
// C column-major (ldc); grid (column tiles, row tiles, splits).  Workgroup
// tile 128 x 256, 8 waves of 64 x 64 (4 x 4 MFMA 16x16x32 tiles), k-step 64.
// The next k-step is prefetched into registers while the current one is
// multiplied from a double-buffered LDS tile; thread t moves chunk t % 8
// of rows (columns) t / 8 + 64 i.  An LDS row holds 64 k values of one row
// of A (column of B) as eight 16-byte chunks, chunk c stored at position
// c ^ (row & 7), so the 16 rows of a fragment read spread over the banks.
// blockIdx.z takes the k range [z kchunk, (z+1) kchunk) and writes its own
// C (offset z * sstride): the partial sums of a split contraction.
constexpr int GB_M = 128, GB_N = 256, GB_K = 64, GB_THREADS = 512;
enum { GOUT_BF16 = 0, GOUT_F32 = 1 };

// wait for this thread's LDS writes (lgkmcnt 0), not for loads in flight
__device__ inline void wait_lds_writes() {
  __builtin_amdgcn_s_waitcnt((3 << 14) | (7 << 4) | 15);   // vmcnt 63, expcnt 7, lgkmcnt 0
}

// multiply the staged k-step from As, Bs into the wave's 64 x 64 tile
__device__ __forceinline__ void bf16_mul(const uint16_t* As, const uint16_t* Bs, int wm, int wn,
                                         int lane, f32x4 (&acc)[4][4]) {
  const int fr = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const int kc = 4 * ks + kq;
    bf16x8 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 64 + i * 16 + fr;
      a[i] = __builtin_bit_cast(bf16x8, *(const uint4*)&As[r * GB_K + 8 * (kc ^ (r & 7))]);
      const int n = wn * 64 + i * 16 + fr;
      b[i] = __builtin_bit_cast(bf16x8, *(const uint4*)&Bs[n * GB_K + 8 * (kc ^ (n & 7))]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

template <int OUT>
__global__ __launch_bounds__(GB_THREADS) void k_gemm_bf16(const uint16_t* __restrict__ A, long long lda,
                                                          const uint16_t* __restrict__ B, long long ldb,
                                                          void* __restrict__ C, long long ldc,
                                                          long long sstride, int kchunk, int K) {
  __shared__ __attribute__((aligned(16))) uint16_t As0[GB_M * GB_K], As1[GB_M * GB_K];
  __shared__ __attribute__((aligned(16))) uint16_t Bs0[GB_N * GB_K], Bs1[GB_N * GB_K];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 2, wn = w & 3;   // 2 x 4 waves
  const long long m0 = (long long)blockIdx.y * GB_M, n0 = (long long)blockIdx.x * GB_N;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(K, k0 + kchunk);
  const int T = (k1 - k0) / GB_K;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // step st multiplies from buffer st % 2 while the loads of step st + 1
  // are in flight; they then go into the other buffer (last read in step
  // st - 1, before the barrier that ended it)
  uint4 ra0, ra1, rb0, rb1, rb2, rb3;
  auto load = [&](int k) {
    const int r = t >> 3, c = t & 7;
    ra0 = *(const uint4*)(A + (m0 + r) * lda + k + 8 * c);
    ra1 = *(const uint4*)(A + (m0 + r + 64) * lda + k + 8 * c);
    rb0 = *(const uint4*)(B + (n0 + r) * ldb + k + 8 * c);
    rb1 = *(const uint4*)(B + (n0 + r + 64) * ldb + k + 8 * c);
    rb2 = *(const uint4*)(B + (n0 + r + 128) * ldb + k + 8 * c);
    rb3 = *(const uint4*)(B + (n0 + r + 192) * ldb + k + 8 * c);
  };
  auto store = [&](uint16_t* As, uint16_t* Bs) {
    const int r = t >> 3, c = t & 7;
    *(uint4*)&As[r * GB_K + 8 * (c ^ (r & 7))] = ra0;
    *(uint4*)&As[(r + 64) * GB_K + 8 * (c ^ (r & 7))] = ra1;
    *(uint4*)&Bs[r * GB_K + 8 * (c ^ (r & 7))] = rb0;
    *(uint4*)&Bs[(r + 64) * GB_K + 8 * (c ^ (r & 7))] = rb1;
    *(uint4*)&Bs[(r + 128) * GB_K + 8 * (c ^ (r & 7))] = rb2;
    *(uint4*)&Bs[(r + 192) * GB_K + 8 * (c ^ (r & 7))] = rb3;
  };
  if (T > 0) {
    load(k0);
    store(As0, Bs0);
  }
  if (T > 1) load(k0 + GB_K);
  wait_lds_writes();
  __builtin_amdgcn_s_barrier();
  for (int st = 0; st < T; st += 2) {
    bf16_mul(As0, Bs0, wm, wn, lane, acc);
    if (st + 1 < T) store(As1, Bs1);
    if (st + 2 < T) load(k0 + (st + 2) * GB_K);
    wait_lds_writes();
    __builtin_amdgcn_s_barrier();
    if (st + 1 >= T) break;
    bf16_mul(As1, Bs1, wm, wn, lane, acc);
    if (st + 2 < T) store(As0, Bs0);
    if (st + 3 < T) load(k0 + (st + 3) * GB_K);
    wait_lds_writes();
    __builtin_amdgcn_s_barrier();
  }
  const int fr = lane & 15;
  // MFMA result: value v of lane l is row 4 (l / 16) + v, column l % 16
  const int rq = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long row = m0 + wm * 64 + i * 16 + rq;
      const long long col = n0 + wn * 64 + j * 16 + fr;
      if constexpr (OUT == GOUT_F32) {
        float* Cf = (float*)C + blockIdx.z * sstride;
        *(f32x4*)(Cf + col * ldc + row) = acc[i][j];
      } else {
        uint16_t* Cb = (uint16_t*)C;
        uint2 pk;
        pk.x = (uint32_t)bf16_of(acc[i][j][0]) | ((uint32_t)bf16_of(acc[i][j][1]) << 16);
        pk.y = (uint32_t)bf16_of(acc[i][j][2]) | ((uint32_t)bf16_of(acc[i][j][3]) << 16);
        *(uint2*)(Cb + col * ldc + row) = pk;
      }
    }
}

// ---- GEMM, FP64 ------------------------------------------------------------------
//
// Same contract in FP64 (A of type TA widened to double while staged).
// Workgroup tile 128 x 64, 4 waves of 64 x 32 (4 x 2 MFMA 16x16x4 tiles),
// k-step 16.  LDS rows have an odd pitch (17 doubles) so the 16 rows a
// fragment read touches fall in distinct banks.
constexpr int GD_M = 128, GD_N = 64, GD_K = 16, GD_PITCH = 17;

template <typename TA>
__global__ __launch_bounds__(256) void k_gemm_f64(const TA* __restrict__ A, long long lda,
                                                  const double* __restrict__ B, long long ldb,
                                                  double* __restrict__ C, long long ldc,
                                                  long long sstride, int kchunk, int K) {
  __shared__ double As[2][GD_M * GD_PITCH];
  __shared__ double Bs[2][GD_N * GD_PITCH];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const long long m0 = (long long)blockIdx.y * GD_M, n0 = (long long)blockIdx.x * GD_N;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(K, k0 + kchunk);
  const int ar = t >> 1, ak = (t & 1) * 8;     // A staging: row, 8 k values
  const int bc = t >> 2, bk = (t & 3) * 4;     // B staging: column, 4 k values
  const TA* Ag = A + (m0 + ar) * lda + ak;
  const double* Bg = B + (n0 + bc) * ldb + bk;
  double ra[8], rb[4];
  f64x4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  auto gload = [&](int k) {
#pragma unroll
    for (int e = 0; e < 8; ++e) ra[e] = (double)Ag[k + e];
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = Bg[k + e];
  };
  auto lstore = [&](int bf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[bf][ar * GD_PITCH + ak + e] = ra[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) Bs[bf][bc * GD_PITCH + bk + e] = rb[e];
  };
  if (k0 < k1) {
    gload(k0);
    lstore(0);
  }
  __syncthreads();
  const int fr = lane & 15, fk = lane >> 4;
  int buf = 0;
  for (int k = k0; k < k1; k += GD_K) {
    const bool more = k + GD_K < k1;
    if (more) gload(k + GD_K);
#pragma unroll
    for (int kk = 0; kk < GD_K; kk += 4) {
      double a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][(wm * 64 + i * 16 + fr) * GD_PITCH + kk + fk];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[buf][(wn * 32 + j * 16 + fr) * GD_PITCH + kk + fk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // FP64 MFMA result: value v of lane l is row l / 16 + 4 v, column l % 16
  double* Cz = C + blockIdx.z * sstride;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long long col = n0 + wn * 32 + j * 16 + fr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long row = m0 + wm * 64 + i * 16 + fk + 4 * v;
        Cz[col * ldc + row] = acc[i][j][v];
      }
    }
}

// ---- GEMM, FP32 operands and accumulation -------------------------------------
//
// The FP64 kernel's tiling with MFMA 16x16x4 FP32: A (FP32 X) as stored, B
// of type TB rounded to FP32 while staged (the FP64 block, or the FP32 U).
template <typename TB>
__global__ __launch_bounds__(256) void k_gemm_f32(const float* __restrict__ A, long long lda,
                                                  const TB* __restrict__ B, long long ldb,
                                                  float* __restrict__ C, long long ldc,
                                                  long long sstride, int kchunk, int K) {
  __shared__ float As[2][GD_M * GD_PITCH];
  __shared__ float Bs[2][GD_N * GD_PITCH];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const long long m0 = (long long)blockIdx.y * GD_M, n0 = (long long)blockIdx.x * GD_N;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(K, k0 + kchunk);
  const int ar = t >> 1, ak = (t & 1) * 8;     // A staging: row, 8 k values
  const int bc = t >> 2, bk = (t & 3) * 4;     // B staging: column, 4 k values
  const float* Ag = A + (m0 + ar) * lda + ak;
  const TB* Bg = B + (n0 + bc) * ldb + bk;
  float ra[8], rb[4];
  f32x4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto gload = [&](int k) {
#pragma unroll
    for (int e = 0; e < 8; ++e) ra[e] = Ag[k + e];
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = (float)Bg[k + e];
  };
  auto lstore = [&](int bf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[bf][ar * GD_PITCH + ak + e] = ra[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) Bs[bf][bc * GD_PITCH + bk + e] = rb[e];
  };
  if (k0 < k1) {
    gload(k0);
    lstore(0);
  }
  __syncthreads();
  const int fr = lane & 15, fk = lane >> 4;
  int buf = 0;
  for (int k = k0; k < k1; k += GD_K) {
    const bool more = k + GD_K < k1;
    if (more) gload(k + GD_K);
#pragma unroll
    for (int kk = 0; kk < GD_K; kk += 4) {
      float a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[buf][(wm * 64 + i * 16 + fr) * GD_PITCH + kk + fk];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[buf][(wn * 32 + j * 16 + fr) * GD_PITCH + kk + fk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // FP32 MFMA result: value v of lane l is row 4 (l / 16) + v, column l % 16
  float* Cz = C + blockIdx.z * sstride;
  const int rq = fk * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long long col = n0 + wn * 32 + j * 16 + fr;
      const long long row = m0 + wm * 64 + i * 16 + rq;
      *(f32x4*)(Cz + col * ldc + row) = acc[i][j];
    }
}

// ---- split-contraction sum with the operator's epilogues -----------------------
//
// t = sum_s part_s (fixed order), then per element (feature j, column c):
// STORE out = t; APPLY out = t + lam p; APPLY_DOT q = t + lam p and <p, q>;
// RESID out = r - (t + lam p); POST z = p + omega (r - (t + lam p)) / D and
// <r, z>; TRUE out = r - (t + lam p) and its squared norm.  Dots leave one
// partial per (column, block) in dots[c * gridDim.x + block].
struct DEpi {
  double* out;
  const double* p;
  const double* r;
  const double* D;
  uint16_t* outb;      // optional BF16 copy of out
  double lam, omega;
  long long ld;        // leading dimension of out, p, r, outb
};

template <int MODE, typename TP>
__global__ __launch_bounds__(256) void k_dreduce(int M, const TP* __restrict__ part, long long ldp,
                                                 long long sstride, int S, DEpi e, double* dots) {
  const int c = blockIdx.y;
  double dot = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = blockIdx.x * 1024 + i * 256 + threadIdx.x;
    if (j >= M) continue;
    const long long po = (long long)c * ldp + j;
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += (double)part[s * sstride + po];
    const long long o = (long long)c * e.ld + j;
    double v;
    if constexpr (MODE == EPI_STORE) {
      v = t;
    } else if constexpr (MODE == EPI_APPLY) {
      v = t + e.lam * e.p[o];
    } else if constexpr (MODE == EPI_APPLY_DOT) {
      const double ps = e.p[o];
      v = t + e.lam * ps;
      dot += ps * v;
    } else if constexpr (MODE == EPI_RESID) {
      v = e.r[o] - (t + e.lam * e.p[o]);
    } else if constexpr (MODE == EPI_POST) {
      const double e2 = e.p[o], rs = e.r[o];
      v = e2 + (e.omega * (rs - (t + e.lam * e2))) / e.D[j];
      dot += rs * v;
    } else {   // EPI_TRUE
      v = e.r[o] - (t + e.lam * e.p[o]);
      dot += v * v;
    }
    e.out[o] = v;
    if (e.outb) e.outb[o] = bf16_of(v);
  }
  if constexpr (MODE == EPI_APPLY_DOT || MODE == EPI_POST || MODE == EPI_TRUE) {
    __shared__ double red[4];
    const double s = block_sum_n<256>(dot, red);
    if (threadIdx.x == 0) dots[c * gridDim.x + blockIdx.x] = s;
  }
}

// ---- block vector kernels (grid: blocks of 1024 features x columns) ------------

// x = 0, r = b, partial ||b||^2
__global__ __launch_bounds__(256) void k_blk_init(int F, long long ld, const double* b, double* x,
                                                  double* r, double* dots) {
  const int c = blockIdx.y;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = blockIdx.x * 1024 + i * 256 + threadIdx.x;
    if (j >= F) continue;
    const long long o = (long long)c * ld + j;
    const double v = b[o];
    x[o] = 0.0;
    r[o] = v;
    s += v * v;
  }
  __shared__ double red[4];
  const double t = block_sum_n<256>(s, red);
  if (threadIdx.x == 0) dots[c * gridDim.x + blockIdx.x] = t;
}

// z = scale r / D (D may be null: z = r); optional BF16 copy; optional <r, z>
__global__ __launch_bounds__(256) void k_blk_diag(int F, long long ld, const double* r, const double* D,
                                                  double scale, double* z, uint16_t* zb, double* dots) {
  const int c = blockIdx.y;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = blockIdx.x * 1024 + i * 256 + threadIdx.x;
    if (j >= F) continue;
    const long long o = (long long)c * ld + j;
    const double rv = r[o];
    const double v = D ? (scale * rv) / D[j] : rv;
    z[o] = v;
    if (zb) zb[o] = bf16_of(v);
    s += rv * v;
  }
  if (dots) {
    __shared__ double red[4];
    const double t = block_sum_n<256>(s, red);
    if (threadIdx.x == 0) dots[c * gridDim.x + blockIdx.x] = t;
  }
}

// p = z + beta_c p; optional BF16 copy
__global__ __launch_bounds__(256) void k_blk_pdir(int F, long long ld, const double* z, double* p,
                                                  uint16_t* pb, const double* beta) {
  const int c = blockIdx.y;
  const double bt = beta[c];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = blockIdx.x * 1024 + i * 256 + threadIdx.x;
    if (j >= F) continue;
    const long long o = (long long)c * ld + j;
    const double v = z[o] + bt * p[o];
    p[o] = v;
    if (pb) pb[o] = bf16_of(v);
  }
}

// x += alpha_c p; r -= alpha_c q; partial ||r||^2
__global__ __launch_bounds__(256) void k_blk_update(int F, long long ld, double* x, double* r,
                                                    const double* p, const double* q,
                                                    const double* alpha, double* dots) {
  const int c = blockIdx.y;
  const double a = alpha[c];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = blockIdx.x * 1024 + i * 256 + threadIdx.x;
    if (j >= F) continue;
    const long long o = (long long)c * ld + j;
    x[o] += a * p[o];
    const double rv = r[o] - a * q[o];
    r[o] = rv;
    s += rv * rv;
  }
  __shared__ double red[4];
  const double t = block_sum_n<256>(s, red);
  if (threadIdx.x == 0) dots[c * gridDim.x + blockIdx.x] = t;
}

// y += x
__global__ void k_blk_add(int F, long long ld, double* y, const double* x) {
  const int c = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) y[(long long)c * ld + j] += x[(long long)c * ld + j];
}

// c_s = scale_s sum_{j in s} v_j  (members in perm[coff[s] .. coff[s+1]))
__global__ void k_blk_restrict(int FC, long long ld, const int* perm, const int* coff,
                               const double* cscale, const double* v, double* cout, long long ldc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (s >= FC) return;
  double t = 0.0;
  for (int e = coff[s]; e < coff[s + 1]; ++e) t += v[(long long)c * ld + perm[e]];
  cout[(long long)c * ldc + s] = cscale[s] * t;
}

// y = Ainv c  (Ainv FC x FC row-major)
__global__ void k_blk_coarse(int FC, const double* Ainv, const double* cin, double* y, long long ldc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= FC) return;
  const double* a = Ainv + (long long)i * FC;
  const double* v = cin + (long long)c * ldc;
  double t = 0.0;
  for (int k = 0; k < FC; ++k) t += a[k] * v[k];
  y[(long long)c * ldc + i] = t;
}

// out = base + scale_{l_j} y_{l_j} (base may be null: 0); optional BF16 copy
__global__ void k_blk_prolong(int F, long long ld, const double* base, const int* labels,
                              const double* cscale, const double* y, long long ldc, double* out,
                              uint16_t* outb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (j >= F) return;
  const long long o = (long long)c * ld + j;
  const int l = labels[j];
  const double v = (base ? base[o] : 0.0) + cscale[l] * y[(long long)c * ldc + l];
  out[o] = v;
  if (outb) outb[o] = bf16_of(v);
}

// additive form: z = omega D^-1 r + P y with <r, z>
__global__ __launch_bounds__(256) void k_blk_additive(int F, long long ld, const double* r,
                                                      const double* D, double omega, const int* labels,
                                                      const double* cscale, const double* y,
                                                      long long ldc, double* z, double* dots) {
  const int c = blockIdx.y;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = blockIdx.x * 1024 + i * 256 + threadIdx.x;
    if (j >= F) continue;
    const long long o = (long long)c * ld + j;
    const int l = labels[j];
    const double rv = r[o];
    const double v = (omega * rv) / D[j] + cscale[l] * y[(long long)c * ldc + l];
    z[o] = v;
    s += rv * v;
  }
  __shared__ double red[4];
  const double t = block_sum_n<256>(s, red);
  if (threadIdx.x == 0) dots[c * gridDim.x + blockIdx.x] = t;
}

// ---- per-column scalars (one block; thread per column) --------------------------

__device__ inline double col_sum(const double* parts, int c, int nb) {
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += parts[c * nb + i];
  return s;
}

// bb_c = ||b_c||^2; a zero column is finished at iteration 0
__global__ void k_col_start(int m, const double* parts, int nb, double* bb, double* rr, int* done,
                            int* iters, int* status, const int* done_in) {
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    const double v = col_sum(parts, c, nb);
    bb[c] = v;
    rr[c] = v;
    const bool fin = (v == 0.0) || (done_in && done_in[c]);
    done[c] = fin ? 1 : 0;
    iters[c] = 0;
    status[c] = fin ? RR_OK : RR_ERR_NOT_CONVERGED;
  }
}

// beta_c = rz_new / rz_old (0 on the first iteration); rz_c = rz_new
__global__ void k_col_beta(int m, const double* parts, int nb, double* rz, double* beta, int first,
                           const int* done, int* status) {
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    const double v = col_sum(parts, c, nb);
    double bt = 0.0;
    if (!first && !done[c]) bt = v / rz[c];
    if (!done[c] && !(v > 0.0 && v < __builtin_inf())) bt = 0.0;
    beta[c] = bt;
    rz[c] = v;
    (void)status;
  }
}

// alpha_c = rz_c / <p, Ap>_c; 0 for finished columns; breakdown ends a column
__global__ void k_col_alpha(int m, const double* parts, int nb, const double* rz, double* alpha,
                            int* done, int* status, int* iters, int it) {
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    const double pq = col_sum(parts, c, nb);
    double a = 0.0;
    if (!done[c]) {
      if (finite_pos(pq) && finite_pos(rz[c])) {
        a = rz[c] / pq;
      } else {
        done[c] = 1;
        status[c] = RR_ERR_BREAKDOWN;
        iters[c] = it;
      }
    }
    alpha[c] = a;
  }
}

// after iteration `it`: rr_c = ||r_c||^2; finish on tol (or at `fixed`);
// nactive = columns still running
__global__ void k_col_check(int m, const double* parts, int nb, const double* bb, double tol2, int it,
                            int fixed, double* rr, int* done, int* iters, int* status, int* nactive) {
  int act = 0;
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    if (done[c]) continue;
    const double v = col_sum(parts, c, nb);
    rr[c] = v;
    iters[c] = it;
    bool fin = false;
    if (!(v == v)) {
      fin = true;
      status[c] = RR_ERR_BREAKDOWN;
    } else if (fixed > 0) {
      if (it >= fixed) {
        fin = true;
        status[c] = RR_OK;
      }
    } else if (v <= tol2 * bb[c]) {
      fin = true;
      status[c] = RR_OK;
    }
    if (fin) done[c] = 1;
    else ++act;
  }
  __shared__ int red[1024 / 64];
  for (int off = 32; off > 0; off >>= 1) act += __shfl_xor(act, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = act;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    *nactive = t;
  }
}

// squared norms per column from partials (host reads the result)
__global__ void k_col_norms(int m, const double* parts, int nb, double* out) {
  for (int c = threadIdx.x; c < m; c += blockDim.x) out[c] = col_sum(parts, c, nb);
}

// ---- setup kernels ------------------------------------------------------------------

// flags: bit 0 non-finite entry, bit 1 negative entry
__global__ void k_dense_scan(long long n, const float* x, int* flags) {
  int f = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float v = x[i];
    if (!(v == v) || v == __builtin_inff() || v == -__builtin_inff()) f |= 1;
    if (v < 0.f) f |= 2;
  }
  if (f) atomicOr(flags, f);
}

// out[c][r] = in[r][c] for an R x C row-major block (both padded), 64 x 64 tiles
__global__ void k_transpose(const float* __restrict__ in, long long ldi, float* __restrict__ out,
                            long long ldo) {
  __shared__ float tile[64][65];
  const long long r0 = (long long)blockIdx.y * 64, c0 = (long long)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 256 threads: 4 rows per pass
  for (int i = ty; i < 64; i += 4) tile[i][tx] = in[(r0 + i) * ldi + c0 + tx];
  __syncthreads();
  for (int i = ty; i < 64; i += 4) out[(c0 + i) * ldo + r0 + tx] = tile[tx][i];
}

__global__ void k_to_bf16_f32(long long n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = bf16_of(x[i]);
}

// BF16 copy of the first F rows of m FP64 columns
__global__ void k_blk_to_bf16(int F, long long ld, const double* x, uint16_t* y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (j < F) y[(long long)c * ld + j] = bf16_of(x[(long long)c * ld + j]);
}

// ||x_j||^2 in FP64 from row j of X^T
__global__ __launch_bounds__(256) void k_dense_colnorm(int N, const float* XT, long long ld, double* c) {
  const float* row = XT + (long long)blockIdx.x * ld;
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) {
    const double v = row[i];
    s += v * v;
  }
  __shared__ double red[4];
  const double t = block_sum_n<256>(s, red);
  if (threadIdx.x == 0) c[blockIdx.x] = t;
}

// Xc[s][i] = scale_s sum_{j in s} X[i][j]  (rows of X^T summed per cluster)
__global__ void k_dense_xc(int N, const float* XT, long long ld, const int* perm, const int* coff,
                           const double* cscale, double* Xc) {
  const int s = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double t = 0.0;
  for (int e = coff[s]; e < coff[s + 1]; ++e) t += (double)XT[(long long)perm[e] * ld + i];
  Xc[(long long)s * ld + i] = cscale[s] * t;
}

__global__ void k_fill_ones(int n, double* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 1.0;
}

__global__ void k_iota(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// ---- host side ------------------------------------------------------------------------

constexpr int kMaxBlockRhs = 4096;
// operator precision of a block application
enum OpPrec { OP_F64 = 0, OP_BF16 = 1, OP_F32 = 2 };

// number of contraction splits: about `target` workgroups, at least 8 k-steps each
void pick_split(int tiles, int K, int bk, int* S, int* kchunk, int target = 1024) {
  const int ktiles = K / bk;
  int s = std::max(1, std::min(cdiv(target, std::max(tiles, 1)), std::max(1, ktiles / 8)));
  const int per = cdiv(ktiles, s);
  *kchunk = per * bk;
  *S = cdiv(ktiles, per);
}

rr_status ensure_dwork(rr_handle* h, int m) {
  DenseX& d = *h->dense;
  if (!h->dwork) {
    h->dwork = new (std::nothrow) DenseWork();
    if (!h->dwork) return fail(RR_ERR_DEVICE, "out of host memory");
  }
  DenseWork& W = *h->dwork;
  const int need = (int)rup(std::max(m, 1), GB_N);
  if (W.m_cap >= need) return RR_OK;
  RR_HIP(hipDeviceSynchronize());
  dense_free_work(W);
  const size_t fp = (size_t)d.Fp * need, np = (size_t)d.Np * need;
  W.m_cap = need;
  W.nb = cdiv(d.F, 1024);
  RR_TRY(zalloc(&W.x, fp)); RR_TRY(zalloc(&W.r, fp)); RR_TRY(zalloc(&W.p, fp));
  RR_TRY(zalloc(&W.q, fp)); RR_TRY(zalloc(&W.z, fp)); RR_TRY(zalloc(&W.e1, fp));
  RR_TRY(zalloc(&W.e2, fp)); RR_TRY(zalloc(&W.rho, fp)); RR_TRY(zalloc(&W.b, fp));
  RR_TRY(zalloc(&W.wx, fp)); RR_TRY(zalloc(&W.wr, fp));
  RR_TRY(zalloc(&W.D, (size_t)d.Fp));
  RR_TRY(zalloc(&W.vb, fp));
  RR_TRY(zalloc(&W.ub, np));
  RR_TRY(zalloc(&W.u, np));
  RR_TRY(zalloc(&W.uf, np));
  // split partials of the column pass (Fp x m_cap per split); the split
  // count is largest when a solve has a single column tile
  int S = 0, kc = 0;
  pick_split(d.Fp / GD_M, d.Np, GD_K, &S, &kc, d.split_target[OP_F64]);
  size_t pb = (size_t)S * fp * sizeof(double);
  pick_split(d.Fp / GD_M, d.Np, GD_K, &S, &kc, d.split_target[OP_F32]);
  pb = std::max(pb, (size_t)S * fp * sizeof(float));
  pick_split(d.Fp / GB_M, d.Np, GB_K, &S, &kc, d.split_target[OP_BF16]);
  pb = std::max(pb, (size_t)S * fp * sizeof(float));
  W.part_bytes = pb;
  RR_HIP(dmalloc(&W.part, pb));
  const int fc = std::max(h->FC, 1);
  RR_TRY(zalloc(&W.c, (size_t)fc * need));
  RR_TRY(zalloc(&W.yc, (size_t)fc * need));
  RR_TRY(zalloc(&W.parts, (size_t)6 * need * W.nb));
  RR_TRY(zalloc(&W.rz, need)); RR_TRY(zalloc(&W.pq, need)); RR_TRY(zalloc(&W.alpha, need));
  RR_TRY(zalloc(&W.beta, need)); RR_TRY(zalloc(&W.rr, need)); RR_TRY(zalloc(&W.bb, need));
  RR_TRY(zalloc(&W.done, need)); RR_TRY(zalloc(&W.iters, need)); RR_TRY(zalloc(&W.status, need));
  RR_TRY(zalloc(&W.done_in, need));
  RR_TRY(zalloc(&W.nactive, 1));
  RR_HIP(hipHostMalloc((void**)&W.nactive_host, sizeof(int), hipHostMallocDefault));
  return RR_OK;
}

}  // namespace

void dense_free_work(DenseWork& W) {
  zfree(W.x); zfree(W.r); zfree(W.p); zfree(W.q); zfree(W.z); zfree(W.e1); zfree(W.e2);
  zfree(W.rho); zfree(W.b); zfree(W.wx); zfree(W.wr); zfree(W.D); zfree(W.vb); zfree(W.ub);
  zfree(W.u); zfree(W.uf); zfree(W.c); zfree(W.yc); zfree(W.parts);
  zfree(W.rz); zfree(W.pq); zfree(W.alpha); zfree(W.beta); zfree(W.rr); zfree(W.bb);
  zfree(W.done); zfree(W.iters); zfree(W.status); zfree(W.done_in); zfree(W.nactive);
  if (W.part) (void)dev_free(W.part);
  W.part = nullptr;
  if (W.nactive_host) (void)hipHostFree(W.nactive_host);
  W.nactive_host = nullptr;
  W.m_cap = 0;
}

void dense_free(rr_handle* h) {
  if (h->dwork) {
    dense_free_work(*h->dwork);
    delete h->dwork;
    h->dwork = nullptr;
  }
  if (h->dense) {
    DenseX& d = *h->dense;
    zfree(d.X32); zfree(d.XT32); zfree(d.Xb); zfree(d.XTb); zfree(d.Xc);
    delete h->dense;
    h->dense = nullptr;
  }
}

namespace {

// ---- operator passes ---------------------------------------------------------------

// U = X V (N x m): FP64 from the FP32 copy, or BF16 (output rounded to BF16)
rr_status pass_rows(rr_handle* h, int m, int op, const double* V, const uint16_t* Vb,
                    hipStream_t s) {
  DenseX& d = *h->dense;
  DenseWork& W = *h->dwork;
  if (op == OP_BF16) {
    const int nt = cdiv(m, GB_N);
    if (d.Np % GB_M || d.Fp % GB_K || nt * GB_N > W.m_cap) return fail(RR_ERR_DEVICE, "internal: GEMM shape");
    dim3 g(nt, d.Np / GB_M, 1);
    k_gemm_bf16<GOUT_BF16><<<g, GB_THREADS, 0, s>>>(d.Xb, d.Fp, Vb, d.Fp, W.ub, d.Np, 0, d.Fp, d.Fp);
  } else {
    const int nt = cdiv(m, GD_N);
    if (d.Np % GD_M || d.Fp % GD_K || nt * GD_N > W.m_cap) return fail(RR_ERR_DEVICE, "internal: GEMM shape");
    dim3 g(nt, d.Np / GD_M, 1);
    if (op == OP_F32)
      k_gemm_f32<double><<<g, 256, 0, s>>>(d.X32, d.Fp, V, d.Fp, W.uf, d.Np, 0, d.Fp, d.Fp);
    else
      k_gemm_f64<float><<<g, 256, 0, s>>>(d.X32, d.Fp, V, d.Fp, W.u, d.Np, 0, d.Fp, d.Fp);
  }
  return RR_OK;
}

// t = X^T U (split contraction) and the epilogue over the first F rows
rr_status pass_cols(rr_handle* h, int m, int op, int mode, const DEpi& e, double* dots,
                    hipStream_t s) {
  DenseX& d = *h->dense;
  DenseWork& W = *h->dwork;
  int S = 0, kc = 0;
  const long long sstride = (long long)d.Fp * W.m_cap;
  dim3 gr(cdiv(d.F, 1024), m);
  if (op == OP_BF16 || op == OP_F32) {
    float* P32 = (float*)W.part;
    if (op == OP_BF16) {
      const int nt = cdiv(m, GB_N);
      pick_split((d.Fp / GB_M) * nt, d.Np, GB_K, &S, &kc, d.split_target[OP_BF16]);
      if (d.Fp % GB_M || d.Np % GB_K || kc % GB_K || (size_t)S * sstride * sizeof(float) > W.part_bytes)
        return fail(RR_ERR_DEVICE, "internal: GEMM shape");
      dim3 g(nt, d.Fp / GB_M, S);
      k_gemm_bf16<GOUT_F32><<<g, GB_THREADS, 0, s>>>(d.XTb, d.Np, W.ub, d.Np, W.part, d.Fp, sstride, kc, d.Np);
    } else {
      const int nt = cdiv(m, GD_N);
      pick_split((d.Fp / GD_M) * nt, d.Np, GD_K, &S, &kc, d.split_target[OP_F32]);
      if (d.Fp % GD_M || d.Np % GD_K || kc % GD_K || (size_t)S * sstride * sizeof(float) > W.part_bytes)
        return fail(RR_ERR_DEVICE, "internal: GEMM shape");
      dim3 g(nt, d.Fp / GD_M, S);
      k_gemm_f32<float><<<g, 256, 0, s>>>(d.XT32, d.Np, W.uf, d.Np, P32, d.Fp, sstride, kc, d.Np);
    }
    const float* P = P32;
    switch (mode) {
      case EPI_STORE: k_dreduce<EPI_STORE, float><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_APPLY: k_dreduce<EPI_APPLY, float><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_APPLY_DOT: k_dreduce<EPI_APPLY_DOT, float><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_RESID: k_dreduce<EPI_RESID, float><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_POST: k_dreduce<EPI_POST, float><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      default: k_dreduce<EPI_TRUE, float><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
    }
  } else {
    const int nt = cdiv(m, GD_N);
    pick_split((d.Fp / GD_M) * nt, d.Np, GD_K, &S, &kc, d.split_target[OP_F64]);
    if (d.Fp % GD_M || d.Np % GD_K || kc % GD_K || (size_t)S * sstride * sizeof(double) > W.part_bytes)
      return fail(RR_ERR_DEVICE, "internal: GEMM shape");
    dim3 g(nt, d.Fp / GD_M, S);
    k_gemm_f64<float><<<g, 256, 0, s>>>(d.XT32, d.Np, W.u, d.Np, (double*)W.part, d.Fp, sstride, kc, d.Np);
    const double* P = (const double*)W.part;
    switch (mode) {
      case EPI_STORE: k_dreduce<EPI_STORE, double><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_APPLY: k_dreduce<EPI_APPLY, double><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_APPLY_DOT: k_dreduce<EPI_APPLY_DOT, double><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_RESID: k_dreduce<EPI_RESID, double><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      case EPI_POST: k_dreduce<EPI_POST, double><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
      default: k_dreduce<EPI_TRUE, double><<<gr, 256, 0, s>>>(d.F, P, d.Fp, sstride, S, e, dots); break;
    }
  }
  return RR_OK;
}

// the operator on block V (FP64, and its BF16 copy Vb for the BF16 form)
rr_status apply(rr_handle* h, int m, int op, const double* V, const uint16_t* Vb, int mode,
                const DEpi& e, double* dots, hipStream_t s) {
  RR_TRY(pass_rows(h, m, op, V, Vb, s));
  return pass_cols(h, m, op, mode, e, dots, s);
}

DEpi epi(const DenseX& d, double* out, const double* p, const double* r, double lam) {
  DEpi e{};
  e.out = out;
  e.p = p;
  e.r = r;
  e.lam = lam;
  e.ld = d.Fp;
  return e;
}

// ---- block PCG ---------------------------------------------------------------------------

struct BlockRun {
  int m = 0;
  int op = OP_F64;                // operator precision
  int kind = RR_PRECOND_VCYCLE;
  double lam = 0.0, omega = 0.0, tol = 1e-10;
  int max_iter = 10000, fixed = 0;
  const LambdaSlot* sl = nullptr;
  const int* done_in = nullptr;   // columns finished before the start
  int applies = 0;
};

// z = B r over the block (with <r, z> partials in dots)
rr_status precond(rr_handle* h, BlockRun& br, const double* r, double* z, double* dots, hipStream_t s) {
  DenseX& d = *h->dense;
  DenseWork& W = *h->dwork;
  const int m = br.m, F = d.F, FC = h->FC;
  dim3 gv(cdiv(F, 1024), m), gf(cdiv(F, kBlock), m), gc(cdiv(std::max(FC, 1), kBlock), m);
  const long long ld = d.Fp;
  switch (br.kind) {
    case RR_PRECOND_NONE:
      k_blk_diag<<<gv, 256, 0, s>>>(F, ld, r, nullptr, 1.0, z, nullptr, dots);
      return RR_OK;
    case RR_PRECOND_JACOBI:
      k_blk_diag<<<gv, 256, 0, s>>>(F, ld, r, W.D, 1.0, z, nullptr, dots);
      return RR_OK;
    case RR_PRECOND_ADDITIVE:
      k_blk_restrict<<<gc, kBlock, 0, s>>>(FC, ld, h->perm, h->coff, h->cscale, r, W.c, FC);
      k_blk_coarse<<<gc, kBlock, 0, s>>>(FC, br.sl->Ainv, W.c, W.yc, FC);
      k_blk_additive<<<gv, 256, 0, s>>>(F, ld, r, W.D, br.omega, h->labels, h->cscale, W.yc, FC, z, dots);
      return RR_OK;
    default: {   // V(1,1)
      uint16_t* vb = br.op == OP_BF16 ? W.vb : nullptr;
      k_blk_diag<<<gv, 256, 0, s>>>(F, ld, r, W.D, br.omega, W.e1, vb, nullptr);
      DEpi e1 = epi(d, W.rho, W.e1, r, br.lam);
      RR_TRY(apply(h, m, br.op, W.e1, W.vb, EPI_RESID, e1, nullptr, s));
      k_blk_restrict<<<gc, kBlock, 0, s>>>(FC, ld, h->perm, h->coff, h->cscale, W.rho, W.c, FC);
      k_blk_coarse<<<gc, kBlock, 0, s>>>(FC, br.sl->Ainv, W.c, W.yc, FC);
      k_blk_prolong<<<gf, kBlock, 0, s>>>(F, ld, W.e1, h->labels, h->cscale, W.yc, FC, W.e2, vb);
      DEpi e2 = epi(d, z, W.e2, r, br.lam);
      e2.D = W.D;
      e2.omega = br.omega;
      RR_TRY(apply(h, m, br.op, W.e2, W.vb, EPI_POST, e2, dots, s));
      br.applies += 2;
      return RR_OK;
    }
  }
}

// PCG from x = 0 on A x = b for every column (b, x: F-blocks).  Per-column
// results in W.iters / W.status / W.rr / W.bb.
rr_status block_pcg(rr_handle* h, BlockRun& br, const double* b, double* x, hipStream_t s) {
  DenseX& d = *h->dense;
  DenseWork& W = *h->dwork;
  const int m = br.m, F = d.F, nb = W.nb;
  const long long ld = d.Fp;
  double* pr_bb = W.parts;
  double* pr_rz = W.parts + (size_t)W.m_cap * nb;
  double* pr_pq = W.parts + (size_t)2 * W.m_cap * nb;
  double* pr_rr = W.parts + (size_t)3 * W.m_cap * nb;
  dim3 gv(cdiv(F, 1024), m);
  const int ct = std::min(1024, (int)rup(m, 64));
  k_blk_init<<<gv, 256, 0, s>>>(F, ld, b, x, W.r, pr_bb);
  k_col_start<<<1, ct, 0, s>>>(m, pr_bb, nb, W.bb, W.rr, W.done, W.iters, W.status, br.done_in);
  const double tol2 = br.tol * br.tol;
  uint16_t* pb = br.op == OP_BF16 ? W.vb : nullptr;
  for (int it = 1; it <= br.max_iter; ++it) {
    RR_TRY(precond(h, br, W.r, W.z, pr_rz, s));
    k_col_beta<<<1, ct, 0, s>>>(m, pr_rz, nb, W.rz, W.beta, it == 1, W.done, W.status);
    k_blk_pdir<<<gv, 256, 0, s>>>(F, ld, W.z, W.p, pb, W.beta);
    DEpi eq = epi(d, W.q, W.p, nullptr, br.lam);
    RR_TRY(apply(h, m, br.op, W.p, W.vb, EPI_APPLY_DOT, eq, pr_pq, s));
    ++br.applies;
    k_col_alpha<<<1, ct, 0, s>>>(m, pr_pq, nb, W.rz, W.alpha, W.done, W.status, W.iters, it);
    k_blk_update<<<gv, 256, 0, s>>>(F, ld, x, W.r, W.p, W.q, W.alpha, pr_rr);
    k_col_check<<<1, ct, 0, s>>>(m, pr_rr, nb, W.bb, tol2, it, br.fixed, W.rr, W.done, W.iters,
                                 W.status, W.nactive);
    RR_HIP(hipMemcpyAsync(W.nactive_host, W.nactive, sizeof(int), hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
    if (*W.nactive_host == 0) break;
  }
  return RR_OK;
}

void copy_block(double* dst, long long ldd, const double* src, long long lds, int rows, int m,
                hipStream_t s, hipError_t* err) {
  *err = hipMemcpy2DAsync(dst, ldd * sizeof(double), src, lds * sizeof(double), rows * sizeof(double),
                          m, hipMemcpyDeviceToDevice, s);
}

}  // namespace

// ---- setup --------------------------------------------------------------------------------

namespace {
std::mutex g_dtune_mu;
std::map<std::string, std::array<int, 3>> g_dtune_cache;
}

// The column pass's split target per operator precision: every candidate
// timed on a block of 256 zero columns (the work does not depend on the
// values), in interleaved rounds, best round each; a candidate must win by
// 3 % to replace the default.  Cached per device and shape bucket.
static rr_status dense_autotune(rr_handle* h, hipStream_t s) {
  DenseX& d = *h->dense;
  int dev = 0;
  RR_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  RR_HIP(hipGetDeviceProperties(&prop, dev));
  auto lg = [](long long v) { int b = 0; while ((1LL << b) < v) ++b; return b; };
  const std::string key = std::string(prop.gcnArchName) + ":" + std::to_string(lg(d.Np)) + ":" +
                          std::to_string(lg(d.Fp));
  {
    std::lock_guard<std::mutex> lk(g_dtune_mu);
    auto it = g_dtune_cache.find(key);
    if (it != g_dtune_cache.end()) {
      for (int k = 0; k < 3; ++k) d.split_target[k] = it->second[k];
      d.split_cached = 1;
      return RR_OK;
    }
  }
  constexpr int kCand = 5, kRounds = 3, kReps = 3, kM = 256;
  const int cand[kCand] = {128, 256, 512, 1024, 2048};
  const int defaults[3] = {d.split_target[0], d.split_target[1], d.split_target[2]};
  for (int k = 0; k < 3; ++k) d.split_target[k] = cand[kCand - 1];
  dense_free_work(*h->dwork);
  RR_TRY(ensure_dwork(h, kM));   // partial buffers for the largest split
  DenseWork& W = *h->dwork;
  hipEvent_t a, b;
  RR_HIP(hipEventCreate(&a));
  RR_HIP(hipEventCreate(&b));
  float best[3][kCand];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < kCand; ++c) best[k][c] = 1e30f;
  rr_status st = RR_OK;
  for (int round = 0; round < kRounds && st == RR_OK; ++round)
    for (int op = 0; op < 3 && st == RR_OK; ++op)
      for (int c = 0; c < kCand && st == RR_OK; ++c) {
        d.split_target[op] = cand[c];
        DEpi e = epi(d, W.q, nullptr, nullptr, 0.0);
        st = pass_rows(h, kM, op, W.p, W.vb, s);
        if (st == RR_OK) st = pass_cols(h, kM, op, EPI_STORE, e, nullptr, s);
        if (st != RR_OK) break;
        if (hipEventRecord(a, s) != hipSuccess) { st = fail(RR_ERR_DEVICE, "autotune event"); break; }
        for (int r = 0; r < kReps && st == RR_OK; ++r) {
          st = pass_rows(h, kM, op, W.p, W.vb, s);
          if (st == RR_OK) st = pass_cols(h, kM, op, EPI_STORE, e, nullptr, s);
        }
        if (st != RR_OK) break;
        float ms = 0.f;
        if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          st = fail(RR_ERR_DEVICE, "autotune timing");
          break;
        }
        best[op][c] = std::min(best[op][c], ms / kReps);
      }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  RR_TRY(st);
  std::array<int, 3> pick{};
  for (int op = 0; op < 3; ++op) {
    int bc = 0;
    for (int c = 0; c < kCand; ++c)
      if (cand[c] == defaults[op]) bc = c;
    for (int c = 0; c < kCand; ++c)
      if (best[op][c] < 0.97f * best[op][bc]) bc = c;
    pick[op] = cand[bc];
    d.split_target[op] = cand[bc];
  }
  dense_free_work(*h->dwork);
  RR_TRY(ensure_dwork(h, 1));
  std::lock_guard<std::mutex> lk(g_dtune_mu);
  g_dtune_cache[key] = pick;
  return RR_OK;
}

rr_status dense_setup(rr_handle* h, const rr_dense* Xin, const rr_setup_opts* o, hipStream_t s) {
  if (!Xin || !Xin->values) return fail(RR_ERR_INVALID_ARG, "null dense matrix");
  if (Xin->n_rows < 1 || Xin->n_cols < 1 || Xin->ld < Xin->n_cols)
    return fail(RR_ERR_INVALID_ARG, "dense X: need n_rows >= 1, n_cols >= 1, ld >= n_cols");
  const long long Np = (long long)rup(Xin->n_rows, kDensePad), Fp = (long long)rup(Xin->n_cols, kDensePad);
  if (Np >= (1ll << 31) || Fp >= (1ll << 31) || Np * Fp >= (1ll << 40))
    return fail(RR_ERR_INVALID_ARG, "dense X too large");
  h->dense = new (std::nothrow) DenseX();
  if (!h->dense) return fail(RR_ERR_DEVICE, "out of host memory");
  DenseX& d = *h->dense;
  d.N = (int)Xin->n_rows;
  d.F = (int)Xin->n_cols;
  d.Np = (int)Np;
  d.Fp = (int)Fp;
  h->X.N = d.N;   // sizes only: the sparse arrays stay empty
  h->X.F = d.F;
  h->w.X = h->X;  // the smoother-weight estimate reads its sizes from work set 0
  const size_t nn = (size_t)Np * Fp;
  RR_TRY(zalloc(&d.X32, nn));
  RR_HIP(hipMemcpy2DAsync(d.X32, Fp * sizeof(float), Xin->values, Xin->ld * sizeof(float),
                          d.F * sizeof(float), d.N, hipMemcpyDeviceToDevice, s));
  int* flags = nullptr;
  RR_TRY(zalloc(&flags, 1));
  k_dense_scan<<<2048, kBlock, 0, s>>>((long long)nn, d.X32, flags);
  int hf = 0;
  RR_HIP(hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  zfree(flags);
  if (hf & 1) return fail(RR_ERR_INVALID_ARG, "dense X has a non-finite entry");
  h->nonneg = !(hf & 2);
  RR_TRY(zalloc(&d.XT32, nn));
  k_transpose<<<dim3(Fp / 64, Np / 64), 256, 0, s>>>(d.X32, Fp, d.XT32, Np);
  RR_TRY(zalloc(&d.Xb, nn));
  RR_TRY(zalloc(&d.XTb, nn));
  k_to_bf16_f32<<<4096, kBlock, 0, s>>>((long long)nn, d.X32, d.Xb);
  k_to_bf16_f32<<<4096, kBlock, 0, s>>>((long long)nn, d.XT32, d.XTb);
  const int F = d.F;
  RR_TRY(zalloc(&h->colnorm, F));
  RR_TRY(zalloc(&h->gersh, F));
  RR_TRY(zalloc(&h->omega_tmp, 1));
  k_dense_colnorm<<<F, 256, 0, s>>>(d.N, d.XT32, Np, h->colnorm);
  RR_TRY(zalloc(&h->fperm, F));
  RR_TRY(zalloc(&h->finv, F));
  k_iota<<<cdiv(F, kBlock), kBlock, 0, s>>>(h->fperm, F);
  k_iota<<<cdiv(F, kBlock), kBlock, 0, s>>>(h->finv, F);
  RR_TRY(ensure_dwork(h, 1));
  if (h->nonneg) {   // g = X^T (X 1)
    DenseWork& W = *h->dwork;
    k_fill_ones<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, W.p);
    RR_TRY(pass_rows(h, 1, OP_F64, W.p, nullptr, s));
    DEpi e = epi(d, W.q, nullptr, nullptr, 0.0);
    RR_TRY(pass_cols(h, 1, OP_F64, EPI_STORE, e, nullptr, s));
    RR_HIP(hipMemcpyAsync(h->gersh, W.q, sizeof(double) * F, hipMemcpyDeviceToDevice, s));
    RR_HIP(hipMemsetAsync(W.p, 0, sizeof(double) * F, s));
  }
  // aggregation
  RR_TRY(zalloc(&h->labels, F));
  const int k = o ? o->n_clusters : 0;
  h->k_req = k;
  const double tk = now_ms();
  if (o && o->labels_in) {
    if (o->n_labels_in < 1) return fail(RR_ERR_INVALID_ARG, "n_labels_in must be >= 1");
    RR_TRY(set_labels(h, o->labels_in, o->n_labels_in, s));
  } else if (k > 0) {
    RR_TRY(zalloc(&h->centres, std::min(k, F)));
    const int mi = (o->kmeans_max_iter > 0) ? o->kmeans_max_iter : 100;
    RR_TRY(dense_kmeans(h, k, o->seed, mi, s));
  }
  h->kmeans_ms = now_ms() - tk;
  if (h->FC > 0) {
    const int fc = h->FC;
    RR_TRY(zalloc(&h->K, (size_t)fc * fc));
    RR_TRY(dense_coarse_gram(h, s));
    const int nslots = (o && o->lambda_slots > 0) ? o->lambda_slots : 4;
    h->slots.resize(nslots);
    for (auto& sl : h->slots) {
      RR_TRY(zalloc(&sl.L, (size_t)fc * fc));
      RR_TRY(zalloc(&sl.Ainv, (size_t)fc * fc));
    }
    RR_TRY(zalloc(&h->chol_work, 2 * (size_t)fc * fc));
    RR_TRY(zalloc(&h->chol_flag, 1));
    // the coarse blocks of the work buffers depend on FC
    dense_free_work(*h->dwork);
    RR_TRY(ensure_dwork(h, 1));
    if (o && o->coarse_eigen) RR_TRY(coarse_eigen(h, &h->eig_sweeps, s));
  }
  if (o && o->autotune) RR_TRY(dense_autotune(h, s));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  return RR_OK;
}

// K = (X P)^T (X P): the coarse columns X P (FP64), then one FP64 GEMM.
// K = Xc Xc^T (fc x fc, ld fc) from Xc (FCp x Np row-major FP64, rows past
// fc and columns past the data zero; FCp a multiple of 128, Np of 16): one
// FP64 matrix-core GEMM split over the contraction, partials added in a
// fixed order.
rr_status gram_rows(const double* Xc, int fc, int FCp, int Np, double* K, hipStream_t s) {
  int S = 0, kc = 0;
  const int tiles = (FCp / GD_M) * cdiv(fc, GD_N);
  pick_split(tiles, Np, GD_K, &S, &kc);
  const long long sstride = (long long)FCp * FCp;
  double* part = nullptr;
  RR_TRY(zalloc(&part, (size_t)S * sstride));
  if (FCp % GD_M || Np % GD_K) return fail(RR_ERR_DEVICE, "internal: GEMM shape");
  dim3 g(cdiv(fc, GD_N), FCp / GD_M, S);
  k_gemm_f64<double><<<g, 256, 0, s>>>(Xc, Np, Xc, Np, part, FCp, sstride, kc, Np);
  DEpi e{};
  e.out = K;
  e.ld = fc;
  k_dreduce<EPI_STORE, double><<<dim3(cdiv(fc, 1024), fc), 256, 0, s>>>(fc, part, FCp, sstride, S, e, nullptr);
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  zfree(part);
  return RR_OK;
}

rr_status dense_coarse_gram(rr_handle* h, hipStream_t s) {
  DenseX& d = *h->dense;
  const int fc = h->FC;
  const int FCp = (int)rup(fc, GD_M);
  zfree(d.Xc);
  RR_TRY(zalloc(&d.Xc, (size_t)FCp * d.Np));
  k_dense_xc<<<dim3(cdiv(d.N, kBlock), fc), kBlock, 0, s>>>(d.N, d.XT32, d.Np, h->perm, h->coff,
                                                            h->cscale, d.Xc);
  return gram_rows(d.Xc, fc, FCp, d.Np, h->K, s);
}

rr_status dense_apply_one(rr_handle* h, const double* v, double lam, double* t, hipStream_t s) {
  RR_TRY(ensure_dwork(h, 1));
  DenseX& d = *h->dense;
  DenseWork& W = *h->dwork;
  RR_HIP(hipMemcpyAsync(W.p, v, sizeof(double) * d.F, hipMemcpyDeviceToDevice, s));
  RR_TRY(pass_rows(h, 1, OP_F64, W.p, nullptr, s));
  DEpi e = epi(d, W.q, W.p, nullptr, lam);
  RR_TRY(pass_cols(h, 1, OP_F64, EPI_APPLY, e, nullptr, s));
  RR_HIP(hipMemcpyAsync(t, W.q, sizeof(double) * d.F, hipMemcpyDeviceToDevice, s));
  return RR_OK;
}

rr_status dense_apply_block(rr_handle* h, double lam, int m, const double* v, int64_t ldv, double* q,
                            int64_t ldq, int precision, hipStream_t s) {
  DenseX& d = *h->dense;
  if (m < 1 || m > kMaxBlockRhs) return fail(RR_ERR_INVALID_ARG, "nrhs must be in [1, 4096]");
  if (!v || !q || ldv < d.F || ldq < d.F) return fail(RR_ERR_INVALID_ARG, "bad block arguments");
  if (precision != RR_PREC_F64 && precision != RR_PREC_BF16_IR && precision != RR_PREC_F32_IR)
    return fail(RR_ERR_INVALID_ARG, "precision must be RR_PREC_F64, RR_PREC_F32_IR or RR_PREC_BF16_IR");
  RR_TRY(ensure_dwork(h, m));
  DenseWork& W = *h->dwork;
  hipError_t err;
  copy_block(W.p, d.Fp, v, ldv, d.F, m, s, &err);
  if (err != hipSuccess) return fail(RR_ERR_DEVICE, hipGetErrorString(err));
  const int op = precision == RR_PREC_BF16_IR ? OP_BF16 : (precision == RR_PREC_F32_IR ? OP_F32 : OP_F64);
  if (op == OP_BF16) k_blk_to_bf16<<<dim3(cdiv(d.F, kBlock), m), kBlock, 0, s>>>(d.F, d.Fp, W.p, W.vb);
  DEpi e = epi(d, W.q, W.p, nullptr, lam);
  RR_TRY(apply(h, m, op, W.p, W.vb, EPI_APPLY, e, nullptr, s));
  copy_block(q, ldq, W.q, d.Fp, d.F, m, s, &err);
  if (err != hipSuccess) return fail(RR_ERR_DEVICE, hipGetErrorString(err));
  return RR_OK;
}

// ---- block solve ---------------------------------------------------------------------------

rr_status dense_solve_block(rr_handle* h, double lam, int m, const double* rhs, int64_t ld_rhs,
                            double* wout, int64_t ld_w, const rr_solve_opts* o, rr_solve_info* info,
                            hipStream_t s) {
  const double t0 = now_ms();
  DenseX& d = *h->dense;
  const int F = d.F, N = d.N;
  if (m < 1 || m > kMaxBlockRhs) return fail(RR_ERR_INVALID_ARG, "nrhs must be in [1, 4096]");
  rr_solve_opts op{};
  if (o) op = *o;
  if (!rhs || !wout) return fail(RR_ERR_INVALID_ARG, "null rhs or w");
  if (ld_rhs < (op.rhs_is_b ? F : N) || ld_w < F) return fail(RR_ERR_INVALID_ARG, "leading dimension too small");
  if (op.x_ref || op.residual_history || op.krylov != RR_KRYLOV_PCG || op.graph || op.profile ||
      op.smoother != RR_SMOOTHER_POINT)
    return fail(RR_ERR_UNSUPPORTED, "block solves take tol, max_iter, fixed_iters, precond, rhs_is_b, "
                                    "omega, precision and inner_tol");
  const int kind = op.precond;
  if (kind != RR_PRECOND_NONE && kind != RR_PRECOND_JACOBI && kind != RR_PRECOND_VCYCLE &&
      kind != RR_PRECOND_ADDITIVE)
    return fail(RR_ERR_INVALID_ARG, "block solves take the none, Jacobi, V(1,1) and additive forms");
  if ((kind == RR_PRECOND_VCYCLE || kind == RR_PRECOND_ADDITIVE) && h->FC == 0)
    return fail(RR_ERR_INVALID_ARG, "two-level preconditioner needs a coarse level (n_clusters > 0)");
  if (op.precision != RR_PREC_F64 && op.precision != RR_PREC_BF16_IR && op.precision != RR_PREC_F32_IR)
    return fail(RR_ERR_INVALID_ARG, "precision must be RR_PREC_F64, RR_PREC_F32_IR or RR_PREC_BF16_IR");
  if (op.max_iter < 0 || op.fixed_iters < 0 || op.tol < 0 || op.inner_tol < 0 || op.inner_tol >= 1)
    return fail(RR_ERR_INVALID_ARG, "bad solve option");
  const bool ir = op.precision != RR_PREC_F64;
  if (ir && op.fixed_iters) return fail(RR_ERR_INVALID_ARG, "fixed_iters is not used with refinement");
  RR_TRY(ensure_dwork(h, m));
  DenseWork& W = *h->dwork;
  hipError_t err;
  // b = X^T y (FP64) or b given
  if (op.rhs_is_b) {
    copy_block(W.b, d.Fp, rhs, ld_rhs, F, m, s, &err);
    if (err != hipSuccess) return fail(RR_ERR_DEVICE, hipGetErrorString(err));
  } else {
    RR_HIP(hipMemsetAsync(W.u, 0, sizeof(double) * d.Np * m, s));
    copy_block(W.u, d.Np, rhs, ld_rhs, N, m, s, &err);
    if (err != hipSuccess) return fail(RR_ERR_DEVICE, hipGetErrorString(err));
    DEpi e = epi(d, W.b, nullptr, nullptr, 0.0);
    RR_TRY(pass_cols(h, m, OP_F64, EPI_STORE, e, nullptr, s));
  }
  BlockRun br;
  br.m = m;
  br.kind = kind;
  br.lam = lam;
  br.omega = op.omega;
  br.tol = op.tol > 0 ? op.tol : 1e-10;
  br.max_iter = op.max_iter > 0 ? op.max_iter : 10000;
  br.fixed = op.fixed_iters;
  double coarse_ms = 0.0;
  LambdaSlot* sl = nullptr;
  struct SlotUse {   // keeps the factor from eviction until the solve returns
    LambdaSlot* sl = nullptr;
    ~SlotUse() { if (sl) sl->in_use--; }
  } use;
  if (kind == RR_PRECOND_VCYCLE || kind == RR_PRECOND_ADDITIVE) {
    const double tc = now_ms();
    RR_TRY(get_slot_dense(h, lam, &sl, s));
    coarse_ms = now_ms() - tc;
    sl->in_use++;
    use.sl = sl;
    if (br.omega == 0.0) br.omega = sl->omega;
  }
  if (!std::isfinite(br.omega) || br.omega < 0.0) return fail(RR_ERR_INVALID_ARG, "omega must be finite and >= 0");
  br.sl = sl;
  launch_colnorm_diag(F, h->colnorm, lam, W.D, s);
  std::vector<int> iters(m, 0), status(m, RR_OK), steps(m, 0);
  std::vector<double> rr(m), bb(m);
  const int nb = W.nb;
  double* pr_tr = W.parts + (size_t)4 * W.m_cap * nb;
  dim3 gv(cdiv(F, 1024), m), gf(cdiv(F, kBlock), m);
  const int ct = std::min(1024, (int)rup(m, 64));
  if (!ir) {
    RR_TRY(block_pcg(h, br, W.b, W.x, s));
    RR_HIP(hipMemcpyAsync(iters.data(), W.iters, sizeof(int) * m, hipMemcpyDeviceToHost, s));
    RR_HIP(hipMemcpyAsync(status.data(), W.status, sizeof(int) * m, hipMemcpyDeviceToHost, s));
    RR_HIP(hipMemcpyAsync(rr.data(), W.rr, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    RR_HIP(hipMemcpyAsync(bb.data(), W.bb, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
  } else {
    // refinement: wx = 0, wr = b; corrections A e = wr by BF16-operand PCG
    const double tol = br.tol;
    const bool f32 = op.precision == RR_PREC_F32_IR;
    const double itol = op.inner_tol > 0 ? op.inner_tol : (f32 ? 1e-5 : 1e-3);
    constexpr int kMaxSteps = 60;
    RR_HIP(hipMemsetAsync(W.wx, 0, sizeof(double) * d.Fp * m, s));
    RR_HIP(hipMemcpyAsync(W.wr, W.b, sizeof(double) * d.Fp * m, hipMemcpyDeviceToDevice, s));
    k_blk_init<<<gv, 256, 0, s>>>(F, d.Fp, W.b, W.x, W.r, pr_tr);   // ||b||^2 (x, r scratch)
    k_col_norms<<<1, ct, 0, s>>>(m, pr_tr, nb, W.pq);
    RR_HIP(hipMemcpyAsync(bb.data(), W.pq, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
    std::vector<int> odone(m, 0);
    for (int c = 0; c < m; ++c) {
      rr[c] = bb[c];
      if (bb[c] == 0.0) odone[c] = 1;
    }
    br.op = f32 ? OP_F32 : OP_BF16;
    br.tol = itol;
    br.fixed = 0;
    for (int step = 0; step < kMaxSteps; ++step) {
      int left = 0;
      for (int c = 0; c < m; ++c) left += !odone[c];
      if (!left) break;
      RR_HIP(hipMemcpyAsync(W.done_in, odone.data(), sizeof(int) * m, hipMemcpyHostToDevice, s));
      br.done_in = W.done_in;
      RR_TRY(block_pcg(h, br, W.wr, W.x, s));   // the correction, in x
      std::vector<int> it_in(m), st_in(m);
      RR_HIP(hipMemcpyAsync(it_in.data(), W.iters, sizeof(int) * m, hipMemcpyDeviceToHost, s));
      RR_HIP(hipMemcpyAsync(st_in.data(), W.status, sizeof(int) * m, hipMemcpyDeviceToHost, s));
      k_blk_add<<<gf, kBlock, 0, s>>>(F, d.Fp, W.wx, W.x);
      // wr = b - A wx (FP64 operator) with its squared norms
      RR_TRY(pass_rows(h, m, OP_F64, W.wx, nullptr, s));
      DEpi e = epi(d, W.wr, W.wx, W.b, lam);
      RR_TRY(pass_cols(h, m, OP_F64, EPI_TRUE, e, pr_tr, s));
      br.applies += 1;
      k_col_norms<<<1, ct, 0, s>>>(m, pr_tr, nb, W.pq);
      RR_HIP(hipMemcpyAsync(rr.data(), W.pq, sizeof(double) * m, hipMemcpyDeviceToHost, s));
      RR_HIP(hipStreamSynchronize(s));
      for (int c = 0; c < m; ++c) {
        if (odone[c]) continue;
        iters[c] += it_in[c];
        steps[c] = step + 1;
        if (!(rr[c] == rr[c])) {
          odone[c] = 1;
          status[c] = RR_ERR_BREAKDOWN;
        } else if (rr[c] <= tol * tol * bb[c]) {
          odone[c] = 1;
          status[c] = RR_OK;
        } else if (iters[c] >= br.max_iter) {
          odone[c] = 1;
          status[c] = RR_ERR_NOT_CONVERGED;
        }
      }
    }
    for (int c = 0; c < m; ++c)
      if (!odone[c]) status[c] = RR_ERR_NOT_CONVERGED;
    RR_HIP(hipMemcpyAsync(W.x, W.wx, sizeof(double) * d.Fp * m, hipMemcpyDeviceToDevice, s));
  }
  // true residual per column
  RR_TRY(pass_rows(h, m, OP_F64, W.x, nullptr, s));
  DEpi et = epi(d, W.q, W.x, W.b, lam);
  RR_TRY(pass_cols(h, m, OP_F64, EPI_TRUE, et, pr_tr, s));
  k_col_norms<<<1, ct, 0, s>>>(m, pr_tr, nb, W.pq);
  std::vector<double> tr(m);
  RR_HIP(hipMemcpyAsync(tr.data(), W.pq, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  copy_block(wout, ld_w, W.x, d.Fp, F, m, s, &err);
  if (err != hipSuccess) return fail(RR_ERR_DEVICE, hipGetErrorString(err));
  RR_HIP(hipStreamSynchronize(s));
  RR_HIP(hipGetLastError());
  const double ms = now_ms() - t0;
  rr_status worst = RR_OK;
  for (int c = 0; c < m; ++c) {
    if (info) {
      rr_solve_info& in = info[c];
      std::memset(&in, 0, sizeof(in));
      in.status = status[c];
      in.iters = iters[c];
      in.op_applies = br.applies;
      in.ir_steps = ir ? steps[c] : 0;
      in.relres = bb[c] > 0 ? std::sqrt(rr[c] / bb[c]) : 0.0;
      in.true_relres = bb[c] > 0 ? std::sqrt(tr[c] / bb[c]) : 0.0;
      in.omega = br.omega;
      in.ms = ms;
      in.coarse_ms = coarse_ms;
      in.fallback_iter = -1;
    }
    if (status[c] == RR_ERR_BREAKDOWN) worst = RR_ERR_BREAKDOWN;
    else if (status[c] == RR_ERR_NOT_CONVERGED && worst == RR_OK) worst = RR_ERR_NOT_CONVERGED;
  }
  if (worst == RR_ERR_NOT_CONVERGED) return fail(worst, "a column reached max_iter before the tolerance");
  if (worst == RR_ERR_BREAKDOWN) return fail(worst, "breakdown in a column: <p,Ap> or <r,z> not positive");
  return RR_OK;
}

// ---- k-means++ over the columns of a dense X (FP64) -----------------------------
//
// The clustering section's K-means++ with Euclidean distances, on the
// columns x_j in R^N.  Seeding: ||x_j - x_c||^2 = c_j + c_c - 2 x_j^T x_c
// (clamped at 0, exactly 0 for j = c), the next centre is the first j whose
// inclusive prefix of D^2 exceeds u T (u the next SplitMix64 draw in [0, 1),
// T the total).  Lloyd: mu_s = mean of the member columns, score_js =
// ||mu_s||^2 - 2 x_j^T mu_s (||x_j||^2 dropped), the lowest s on ties, stop
// when no label changes.  Sums run in FP64 in another order than a CPU
// implementation, so labels agree with one up to near-ties.

namespace {

struct SeedState {
  int stop;        // T = 0 reached: no further centre
  int n_centres;
  int last;        // the newest centre
  int pad;
};

// d2_j = min(d2_j, c_j + c_c - 2 x_j^T x_c) for the newest centre c
// (first = 1: d2_j = that distance).  One wave per feature.
__global__ __launch_bounds__(256) void k_km_dist(int F, int N, const float* __restrict__ XT, long long ld,
                                                 const double* __restrict__ cn, const SeedState* st,
                                                 double* __restrict__ d2, int first) {
  if (st->stop) return;
  const int c = st->last;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= F) return;
  const float* xj = XT + (long long)j * ld;
  const float* xc = XT + (long long)c * ld;
  double g = 0.0;
  for (int i = lane; i < N; i += 64) g += (double)xj[i] * (double)xc[i];
  for (int off = 32; off > 0; off >>= 1) g += __shfl_xor(g, off, 64);
  if (lane == 0) {
    double d = (j == c) ? 0.0 : cn[j] + cn[c] - 2.0 * g;
    if (d < 0.0) d = 0.0;
    d2[j] = first ? d : fmin(d2[j], d);
  }
}

// One block: T = sum d2 (chunks in a fixed order), r = u T, and the first j
// whose inclusive prefix exceeds r becomes centre `slot`; T = 0 stops the
// seeding.
constexpr int kDrawThreads = 1024;
__global__ __launch_bounds__(kDrawThreads) void k_km_draw(int F, const double* __restrict__ d2,
                                                          const double* __restrict__ u, int slot,
                                                          int* centres, SeedState* st) {
  __shared__ double pre[kDrawThreads];
  __shared__ double total;
  __shared__ int pick, stopped;
  const int t = threadIdx.x;
  if (t == 0) {
    stopped = st->stop;
    pick = F;
  }
  __syncthreads();
  if (stopped) return;
  const int L = (F + kDrawThreads - 1) / kDrawThreads;
  const int j0 = min(F, t * L), j1 = min(F, j0 + L);
  double sum = 0.0;
  for (int j = j0; j < j1; ++j) sum += d2[j];
  pre[t] = sum;
  __syncthreads();
  if (t == 0) {   // exclusive prefix of the chunk sums, in chunk order
    double run = 0.0;
    for (int i = 0; i < kDrawThreads; ++i) {
      const double v = pre[i];
      pre[i] = run;
      run += v;
    }
    total = run;
  }
  __syncthreads();
  if (!(total > 0.0)) {
    if (t == 0) st->stop = 1;
    return;
  }
  const double r = u[slot - 1] * total;
  double run = pre[t];
  for (int j = j0; j < j1; ++j) {
    const double nx = run + d2[j];
    if (nx > r && run <= r) atomicMin(&pick, j);
    run = nx;
  }
  __syncthreads();
  if (t == 0) {
    const int j = min(pick, F - 1);
    centres[slot] = j;
    st->last = j;
    st->n_centres = slot + 1;
  }
}

__global__ void k_km_first(int c, int* centres, SeedState* st) {
  centres[0] = c;
  st->stop = 0;
  st->n_centres = 1;
  st->last = c;
}

// labels: centre s -> s, every other feature -1
__global__ void k_km_init_labels(int F, int* labels) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < F) labels[j] = -1;
}
__global__ void k_km_set_centres(int nc, const int* centres, int* labels) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nc) labels[centres[s]] = s;
}

// mu[s][i] = (1 / n_s) sum_{j in s} X[i][j]  (rows of X^T); ||mu_s||^2 later
__global__ void k_km_means(int N, const float* XT, long long ld, const int* perm, const int* off,
                           double* mu) {
  const int s = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int a = off[s], b = off[s + 1];
  double t = 0.0;
  for (int e = a; e < b; ++e) t += (double)XT[(long long)perm[e] * ld + i];
  mu[(long long)s * ld + i] = (b > a) ? t / (double)(b - a) : 0.0;
}

__global__ __launch_bounds__(256) void k_km_norms(int N, const double* mu, long long ld, double* q) {
  const double* m = mu + (long long)blockIdx.x * ld;
  double v = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) v += m[i] * m[i];
  __shared__ double red[4];
  const double t = block_sum_n<256>(v, red);
  if (threadIdx.x == 0) q[blockIdx.x] = t;
}

// new label = argmin over active s of q_s - 2 G_js (lowest s on ties);
// counts changes
__global__ void k_km_assign(int F, int k, const double* __restrict__ G, long long ldg,
                            const double* __restrict__ q, const int* __restrict__ off, int* labels,
                            int* changed) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F) return;
  double best = __builtin_inf();
  int bs = -1;
  for (int s2 = 0; s2 < k; ++s2) {
    if (off[s2 + 1] == off[s2]) continue;
    const double v = q[s2] - 2.0 * G[(long long)s2 * ldg + j];
    if (v < best) {
      best = v;
      bs = s2;
    }
  }
  if (bs != labels[j]) {
    labels[j] = bs;
    atomicAdd(changed, 1);
  }
}

}  // namespace

rr_status dense_kmeans(rr_handle* h, int k, uint64_t seed, int max_iter, hipStream_t s) {
  DenseX& d = *h->dense;
  const int F = d.F, N = d.N;
  k = std::min(k, F);
  // seeding draws (host SplitMix64, as many as the seeding can use)
  uint64_t st_rng = seed;
  const int first = (int)(splitmix64_next(st_rng) % (uint64_t)F);
  std::vector<double> u(std::max(k - 1, 1));
  for (int i = 0; i + 1 < k; ++i) u[i] = (double)(splitmix64_next(st_rng) >> 11) * (1.0 / 9007199254740992.0);
  double *d2 = nullptr, *du = nullptr;
  SeedState* st = nullptr;
  RR_TRY(zalloc(&d2, F));
  RR_TRY(zalloc(&du, u.size()));
  RR_TRY(zalloc(&st, 1));
  RR_HIP(hipMemcpyAsync(du, u.data(), sizeof(double) * u.size(), hipMemcpyHostToDevice, s));
  k_km_first<<<1, 1, 0, s>>>(first, h->centres, st);
  const int gd = cdiv(F, 4);
  k_km_dist<<<gd, 256, 0, s>>>(F, N, d.XT32, d.Np, h->colnorm, st, d2, 1);
  for (int slot = 1; slot < k; ++slot) {
    k_km_draw<<<1, kDrawThreads, 0, s>>>(F, d2, du, slot, h->centres, st);
    if (slot + 1 < k) k_km_dist<<<gd, 256, 0, s>>>(F, N, d.XT32, d.Np, h->colnorm, st, d2, 0);
  }
  SeedState hs{};
  RR_HIP(hipMemcpyAsync(&hs, st, sizeof(SeedState), hipMemcpyDeviceToHost, s));
  RR_HIP(hipStreamSynchronize(s));
  zfree(d2);
  zfree(du);
  zfree(st);
  const int nc = hs.n_centres;
  h->n_centres = nc;
  // Lloyd
  const int kp = (int)rup(nc, GD_N);
  double *mu = nullptr, *q = nullptr, *G = nullptr, *part = nullptr;
  int *labels = h->labels, *perm = nullptr, *off = nullptr, *changed = nullptr;
  RR_TRY(zalloc(&mu, (size_t)kp * d.Np));
  RR_TRY(zalloc(&q, kp));
  RR_TRY(zalloc(&G, (size_t)kp * d.Fp));
  RR_TRY(zalloc(&perm, F));
  RR_TRY(zalloc(&off, nc + 1));
  RR_TRY(zalloc(&changed, 1));
  int S = 0, kc = 0;
  pick_split((d.Fp / GD_M) * (kp / GD_N), d.Np, GD_K, &S, &kc);
  const long long sstride = (long long)d.Fp * kp;
  RR_TRY(zalloc(&part, (size_t)S * sstride));
  k_km_init_labels<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, labels);
  k_km_set_centres<<<cdiv(nc, kBlock), kBlock, 0, s>>>(nc, h->centres, labels);
  std::vector<int> hl(F), hperm(F), hoff(nc + 1);
  int it = 0;
  rr_status res = RR_OK;
  while (it < max_iter) {
    // members per cluster (host counting sort of F labels)
    RR_HIP(hipMemcpyAsync(hl.data(), labels, sizeof(int) * F, hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
    std::fill(hoff.begin(), hoff.end(), 0);
    for (int j = 0; j < F; ++j)
      if (hl[j] >= 0) ++hoff[hl[j] + 1];
    for (int c = 0; c < nc; ++c) hoff[c + 1] += hoff[c];
    {
      std::vector<int> pos(hoff.begin(), hoff.end() - 1);
      for (int j = 0; j < F; ++j)
        if (hl[j] >= 0) hperm[pos[hl[j]]++] = j;
    }
    RR_HIP(hipMemcpyAsync(perm, hperm.data(), sizeof(int) * F, hipMemcpyHostToDevice, s));
    RR_HIP(hipMemcpyAsync(off, hoff.data(), sizeof(int) * (nc + 1), hipMemcpyHostToDevice, s));
    k_km_means<<<dim3(cdiv(N, kBlock), nc), kBlock, 0, s>>>(N, d.XT32, d.Np, perm, off, mu);
    k_km_norms<<<nc, 256, 0, s>>>(N, mu, d.Np, q);
    // G = X^T mu  (F x nc, FP64 matrix cores)
    if (d.Fp % GD_M || d.Np % GD_K || kc % GD_K) {
      res = fail(RR_ERR_DEVICE, "internal: GEMM shape");
      break;
    }
    k_gemm_f64<float><<<dim3(kp / GD_N, d.Fp / GD_M, S), 256, 0, s>>>(d.XT32, d.Np, mu, d.Np, part, d.Fp,
                                                                        sstride, kc, d.Np);
    DEpi e{};
    e.out = G;
    e.ld = d.Fp;
    k_dreduce<EPI_STORE, double><<<dim3(cdiv(F, 1024), nc), 256, 0, s>>>(F, part, d.Fp, sstride, S, e, nullptr);
    RR_HIP(hipMemsetAsync(changed, 0, sizeof(int), s));
    k_km_assign<<<cdiv(F, kBlock), kBlock, 0, s>>>(F, nc, G, d.Fp, q, off, labels, changed);
    int hc = 0;
    RR_HIP(hipMemcpyAsync(&hc, changed, sizeof(int), hipMemcpyDeviceToHost, s));
    RR_HIP(hipStreamSynchronize(s));
    ++it;
    if (hc == 0) break;
  }
  h->kmeans_iters = it;
  zfree(mu); zfree(q); zfree(G); zfree(part); zfree(perm); zfree(off); zfree(changed);
  RR_TRY(res);
  // compaction (drop empty clusters), P and the cluster-sorted permutation
  return set_labels(h, h->labels, nc, s);
}

}  // namespace rr
