// The learned coarse correction: a three-layer perceptron (in = F_C + 1,
// two ReLU layers of H units, out = F_C) whose products run on the matrix
// cores in BF16 with FP32 accumulation.  Master weights, Adam moments,
// biases and every reduction are FP32.  Batch-major layout: a batch of B
// inputs is a row-major [B, in] matrix; W1 [H, in], W2 [H, H], W3 [out, H].
#include <cstring>

#include "rr_device.h"

namespace rr {

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// Round to nearest even (finite inputs), as stored in a bf16 operand.
__device__ inline uint16_t f32_to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

// Epilogues of the GEMM C = op(A) op(B) (per element m, n):
enum GemmEpi {
  GE_STORE = 0,       // C32 = acc
  GE_BIAS = 1,        // C32 = acc + bias[n]
  GE_BIAS_RELU = 2,   // C32 = z = acc + bias[n]; C16 = relu(z)
  GE_MASK = 3         // C32 = acc * [Z[m, n] > 0]; C16 = the same in bf16
};

// One wave per 16x16 tile of C; a block of 4 waves covers 32 x 32.  The
// 16x16x16 BF16 matrix instruction takes, in lane l, A[row l%16][k 4(l/16)+i]
// and B[k 4(l/16)+i][col l%16] (i < 4) and returns C[row 4(l/16)+v][col l%16]
// (v < 4).  op(A)[m, k] = transA ? A[k lda + m] : A[m lda + k]; the same for B.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A,
                                                    int lda, int transA,
                                                    const uint16_t* __restrict__ B, int ldb,
                                                    int transB, const float* __restrict__ bias,
                                                    const float* __restrict__ Z,
                                                    float* __restrict__ C32,
                                                    uint16_t* __restrict__ C16, int ldc) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int m0 = blockIdx.y * 32 + (wave >> 1) * 16;
  const int n0 = blockIdx.x * 32 + (wave & 1) * 16;
  if (m0 >= M || n0 >= N) return;
  const int ar = m0 + (l & 15), bc = n0 + (l & 15), kq = 4 * (l >> 4);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + kq + i;
      uint16_t av = 0, bv = 0;
      if (ar < M && k < K) av = transA ? A[(size_t)k * lda + ar] : A[(size_t)ar * lda + k];
      if (bc < N && k < K) bv = transB ? B[(size_t)bc * ldb + k] : B[(size_t)k * ldb + bc];
      a[i] = (short)av;
      b[i] = (short)bv;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = m0 + 4 * (l >> 4) + v, n = n0 + (l & 15);
    if (m >= M || n >= N) continue;
    const size_t o = (size_t)m * ldc + n;
    float c = acc[v];
    if constexpr (EPI == GE_BIAS) c += bias[n];
    if constexpr (EPI == GE_BIAS_RELU) {
      c += bias[n];
      C16[o] = f32_to_bf16(c > 0.f ? c : 0.f);
    }
    if constexpr (EPI == GE_MASK) {
      c = (Z[o] > 0.f) ? c : 0.f;
      C16[o] = f32_to_bf16(c);
    }
    C32[o] = c;
  }
}

template <int EPI>
static void gemm(int M, int N, int K, const uint16_t* A, int lda, int transA, const uint16_t* B,
                 int ldb, int transB, const float* bias, const float* Z, float* C32, uint16_t* C16,
                 int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  dim3 grid(cdiv(N, 32), cdiv(M, 32));
  k_gemm_bf16<EPI><<<grid, 256, 0, s>>>(M, N, K, A, lda, transA, B, ldb, transB, bias, Z, C32, C16,
                                        ldc);
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f32_to_bf16(x[i]);
}
static void to_bf16(const float* x, uint16_t* y, long long n, hipStream_t s) {
  if (n > 0) k_to_bf16<<<cdiv(n, kBlock), kBlock, 0, s>>>(x, y, n);
}

// column sums over the batch: g[n] = sum_b G[b, n] (fixed order)
__global__ void k_colsum(int Bn, int N, const float* __restrict__ G, float* __restrict__ g) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int b = 0; b < Bn; ++b) s += G[(size_t)b * N + n];
  g[n] = s;
}

// dY = (Y - T) / B in FP32 and BF16; per-row squared errors for the loss
__global__ void k_loss_grad(int Bn, int N, const float* __restrict__ Y, const float* __restrict__ T,
                            const int* __restrict__ rows, float* __restrict__ dY32,
                            uint16_t* __restrict__ dY16, float* __restrict__ err2) {
  const int b = blockIdx.x;
  const int t = rows ? rows[b] : b;
  float e = 0.f;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const float d = Y[(size_t)b * N + n] - T[(size_t)t * N + n];
    e += d * d;
    const float g = d / (float)Bn;
    dY32[(size_t)b * N + n] = g;
    dY16[(size_t)b * N + n] = f32_to_bf16(g);
  }
  __shared__ double red[kBlock / 64];
  const double tot = block_sum((double)e, red);
  if (threadIdx.x == 0) err2[b] = (float)tot;
}

// gather a mini-batch of inputs (FP32 rows) into BF16
__global__ void k_gather_rows(int Bn, int In, const float* __restrict__ X, const int* __restrict__ rows,
                              uint16_t* __restrict__ Xb) {
  const int b = blockIdx.x;
  const int t = rows ? rows[b] : b;
  for (int k = threadIdx.x; k < In; k += blockDim.x) Xb[(size_t)b * In + k] = f32_to_bf16(X[(size_t)t * In + k]);
}

// Adam with bias correction on the FP32 master weights, then their BF16 copy
__global__ void k_adam(long long n, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, uint16_t* __restrict__ w16,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  w16[i] = f32_to_bf16(wi);
}

// ---- network storage ---------------------------------------------------------

void Mlp::offsets(size_t* o) const {
  o[0] = 0;                                   // W1
  o[1] = o[0] + (size_t)hid * in;             // b1
  o[2] = o[1] + hid;                          // W2
  o[3] = o[2] + (size_t)hid * hid;            // b2
  o[4] = o[3] + hid;                          // W3
  o[5] = o[4] + (size_t)out * hid;            // b3
  o[6] = o[5] + out;                          // end
}

void free_mlp(Mlp& n) {
  for (void* p : {(void*)n.w, (void*)n.w16, (void*)n.m, (void*)n.v, (void*)n.g, (void*)n.xb,
                  (void*)n.z1, (void*)n.a1, (void*)n.z2, (void*)n.a2, (void*)n.y, (void*)n.dy32,
                  (void*)n.dy16, (void*)n.dz2, (void*)n.dz2b, (void*)n.dz1, (void*)n.dz1b,
                  (void*)n.err2, (void*)n.rows})
    if (p) (void)dev_free(p);
  n = Mlp{};
}

template <typename T>
static rr_status mal(T** p, size_t n) {
  *p = nullptr;
  hipError_t e = dmalloc((void**)p, sizeof(T) * (n ? n : 1));
  if (e != hipSuccess) return fail(RR_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  return RR_OK;
}

rr_status mlp_alloc(Mlp& n, int in, int hid, int out, int max_batch) {
  free_mlp(n);
  n.in = in;
  n.hid = hid;
  n.out = out;
  n.max_batch = max_batch;
  size_t o[7];
  n.offsets(o);
  n.nparam = o[6];
  RR_TRY(mal(&n.w, n.nparam));
  RR_TRY(mal(&n.w16, n.nparam));
  RR_TRY(mal(&n.m, n.nparam));
  RR_TRY(mal(&n.v, n.nparam));
  RR_TRY(mal(&n.g, n.nparam));
  const size_t B = max_batch;
  RR_TRY(mal(&n.xb, B * in));
  RR_TRY(mal(&n.z1, B * hid));
  RR_TRY(mal(&n.a1, B * hid));
  RR_TRY(mal(&n.z2, B * hid));
  RR_TRY(mal(&n.a2, B * hid));
  RR_TRY(mal(&n.y, B * out));
  RR_TRY(mal(&n.dy32, B * out));
  RR_TRY(mal(&n.dy16, B * out));
  RR_TRY(mal(&n.dz2, B * hid));
  RR_TRY(mal(&n.dz2b, B * hid));
  RR_TRY(mal(&n.dz1, B * hid));
  RR_TRY(mal(&n.dz1b, B * hid));
  RR_TRY(mal(&n.err2, B));
  RR_TRY(mal(&n.rows, B));
  return RR_OK;
}

rr_status mlp_set(Mlp& n, const float* host, hipStream_t s) {
  RR_HIP(hipMemcpyAsync(n.w, host, sizeof(float) * n.nparam, hipMemcpyHostToDevice, s));
  to_bf16(n.w, n.w16, (long long)n.nparam, s);
  RR_HIP(hipMemsetAsync(n.m, 0, sizeof(float) * n.nparam, s));
  RR_HIP(hipMemsetAsync(n.v, 0, sizeof(float) * n.nparam, s));
  n.t = 0;
  RR_HIP(hipStreamSynchronize(s));
  return RR_OK;
}

// forward of the first Bn rows of n.xb (BF16 inputs) into n.y
void mlp_forward(Mlp& n, int Bn, hipStream_t s) {
  size_t o[7];
  n.offsets(o);
  gemm<GE_BIAS_RELU>(Bn, n.hid, n.in, n.xb, n.in, 0, n.w16 + o[0], n.in, 1, n.w + o[1], nullptr,
                     n.z1, n.a1, n.hid, s);
  gemm<GE_BIAS_RELU>(Bn, n.hid, n.hid, n.a1, n.hid, 0, n.w16 + o[2], n.hid, 1, n.w + o[3], nullptr,
                     n.z2, n.a2, n.hid, s);
  gemm<GE_BIAS>(Bn, n.out, n.hid, n.a2, n.hid, 0, n.w16 + o[4], n.hid, 1, n.w + o[5], nullptr, n.y,
                nullptr, n.out, s);
}

// gradients into n.g from dY (n.dy32 / n.dy16) after mlp_forward
void mlp_backward(Mlp& n, int Bn, hipStream_t s) {
  size_t o[7];
  n.offsets(o);
  // layer 3
  gemm<GE_STORE>(n.out, n.hid, Bn, n.dy16, n.out, 1, n.a2, n.hid, 0, nullptr, nullptr, n.g + o[4],
                 nullptr, n.hid, s);
  k_colsum<<<cdiv(n.out, kBlock), kBlock, 0, s>>>(Bn, n.out, n.dy32, n.g + o[5]);
  gemm<GE_MASK>(Bn, n.hid, n.out, n.dy16, n.out, 0, n.w16 + o[4], n.hid, 0, nullptr, n.z2, n.dz2,
                n.dz2b, n.hid, s);
  // layer 2
  gemm<GE_STORE>(n.hid, n.hid, Bn, n.dz2b, n.hid, 1, n.a1, n.hid, 0, nullptr, nullptr, n.g + o[2],
                 nullptr, n.hid, s);
  k_colsum<<<cdiv(n.hid, kBlock), kBlock, 0, s>>>(Bn, n.hid, n.dz2, n.g + o[3]);
  gemm<GE_MASK>(Bn, n.hid, n.hid, n.dz2b, n.hid, 0, n.w16 + o[2], n.hid, 0, nullptr, n.z1, n.dz1,
                n.dz1b, n.hid, s);
  // layer 1
  gemm<GE_STORE>(n.hid, n.in, Bn, n.dz1b, n.hid, 1, n.xb, n.in, 0, nullptr, nullptr, n.g + o[0],
                 nullptr, n.in, s);
  k_colsum<<<cdiv(n.hid, kBlock), kBlock, 0, s>>>(Bn, n.hid, n.dz1, n.g + o[1]);
}

void mlp_load_inputs(Mlp& n, const float* X, const int* rows, int Bn, hipStream_t s) {
  k_gather_rows<<<Bn, kBlock, 0, s>>>(Bn, n.in, X, rows, n.xb);
}

void mlp_set_dout(Mlp& n, const float* dY, int Bn, hipStream_t s) {
  RR_HIP_VOID(hipMemcpyAsync(n.dy32, dY, sizeof(float) * (size_t)Bn * n.out, hipMemcpyDeviceToDevice, s));
  to_bf16(n.dy32, n.dy16, (long long)Bn * n.out, s);
}

void mlp_loss_grad(Mlp& n, const float* T, const int* rows, int Bn, hipStream_t s) {
  k_loss_grad<<<Bn, kBlock, 0, s>>>(Bn, n.out, n.y, T, rows, n.dy32, n.dy16, n.err2);
}

void mlp_adam(Mlp& n, float lr, hipStream_t s) {
  n.t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)n.t), c2 = 1.f - powf(b2, (float)n.t);
  k_adam<<<cdiv((long long)n.nparam, kBlock), kBlock, 0, s>>>((long long)n.nparam, n.w, n.g, n.m,
                                                              n.v, n.w16, lr, b1, b2, 1e-8f, c1, c2);
}

// Network input of the learned coarse correction for one residual: with
// c = P^T r, xb = bf16([c / ||c||, log lambda]) and scale = ||c|| (one block).
__global__ __launch_bounds__(kBlock) void k_learned_in(int FC, const double* __restrict__ c,
                                                       double loglam, uint16_t* __restrict__ xb,
                                                       double* __restrict__ scale, const int* done) {
  if (is_done(done)) return;
  __shared__ double red[kBlock / 64];
  double s2 = 0.0;
  for (int i = threadIdx.x; i < FC; i += kBlock) s2 += c[i] * c[i];
  const double nrm = sqrt(block_sum(s2, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < FC; i += kBlock) xb[i] = f32_to_bf16((float)(c[i] * inv));
  if (threadIdx.x == 0) {
    xb[FC] = f32_to_bf16((float)loglam);
    *scale = nrm;
  }
}

void launch_learned_in(int FC, const double* c, double lam, uint16_t* xb, double* scale,
                       const int* done, hipStream_t s) {
  k_learned_in<<<1, kBlock, 0, s>>>(FC, c, log(lam), xb, scale, done);
}

// yc_i = ||c|| y_i / (K_ii + lambda) (FP64): the network predicts the coarse
// correction in units of the coarse Jacobi step, so that its outputs are of
// order one whatever the scale of A_c
__global__ void k_learned_out(int FC, const float* __restrict__ y, const double* __restrict__ scale,
                              const double* __restrict__ K, double lam, double* __restrict__ yc,
                              const int* done) {
  if (is_done(done)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < FC) yc[i] = *scale * (double)y[i] / (K[(size_t)i * FC + i] + lam);
}

void launch_learned_out(int FC, const float* y, const double* scale, const double* K, double lam, double* yc,
                        const int* done, hipStream_t s) {
  k_learned_out<<<cdiv(FC, kBlock), kBlock, 0, s>>>(FC, y, scale, K, lam, yc, done);
}

// Training pairs from coarse residual snapshots: for pair q with r_c = S[q],
// input [r_c/||r_c||, log lambda] and target (K_ii + lambda) (A_c^-1 r_c)_i /
// ||r_c|| (the coarse correction in units of the coarse Jacobi step), where
// Ainv_rc[q] = A_c^-1 r_c has been formed already (one block per pair).
__global__ __launch_bounds__(kBlock) void k_make_pairs(int FC, const double* __restrict__ S,
                                                       const double* __restrict__ Ainv_rc,
                                                       const double* __restrict__ K, double lam,
                                                       double loglam, float* __restrict__ inputs,
                                                       float* __restrict__ targets) {
  const int q = blockIdx.x;
  const double* rc = S + (size_t)q * FC;
  __shared__ double red[kBlock / 64];
  double s2 = 0.0;
  for (int i = threadIdx.x; i < FC; i += kBlock) s2 += rc[i] * rc[i];
  const double nrm = sqrt(block_sum(s2, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  float* in = inputs + (size_t)q * (FC + 1);
  float* tg = targets + (size_t)q * FC;
  for (int i = threadIdx.x; i < FC; i += kBlock) {
    in[i] = (float)(rc[i] * inv);
    tg[i] = (float)(Ainv_rc[(size_t)q * FC + i] * inv * (K[(size_t)i * FC + i] + lam));
  }
  if (threadIdx.x == 0) in[FC] = (float)loglam;
}

void launch_make_pairs(int FC, int npairs, const double* S, const double* Ainv_rc, const double* K, double lam,
                       float* inputs, float* targets, hipStream_t s) {
  if (npairs > 0)
    k_make_pairs<<<npairs, kBlock, 0, s>>>(FC, S, Ainv_rc, K, lam, log(lam), inputs, targets);
}

}  // namespace rr
