// Learned warm start of the qsGW iteration: per-state features, a
// 16 -> 128 -> 128 -> 1 GELU network (FP32 master weights) with its forward
// pass, MSE gradient and Adam update, and the shifted, re-sorted starting
// orbitals.  The 128-wide layers run on the FP32 matrix-core GEMM engine; the
// rest are element-wise kernels and fixed-order reductions (deterministic).
#include "internal.hpp"

#include <algorithm>

namespace {

constexpr int kIn = 16, kHid = 128;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid,
                  kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid,
                  kNParams = kOffB3 + 1;
static_assert(kNParams == QSGW_MLP_NPARAMS, "parameter layout");

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z = v + b[n] (kept for the backward pass), A = gelu(Z).
struct EpiBiasGelu {
  const float* b;
  float* Z;
  float* A;
  int64_t ld;
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t m, int64_t n, double v,
                                             bool) const {
    const float z = (float)v + b[n];
    if (Z) Z[m * ld + n] = z;
    A[m * ld + n] = gelu(z);
  }
};

// dZ = v * gelu'(Z)
struct EpiGeluGrad {
  const float* Z;
  float* dZ;
  int64_t ld;
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t m, int64_t n, double v,
                                             bool) const {
    dZ[m * ld + n] = (float)v * gelu_grad(Z[m * ld + n]);
  }
};

// Output layer, one wave per row: y = A2 . w3 + b3; with a target also
// dy = 2 (y - t) / n and the squared error (double) for the loss.
__global__ void k_mlp_out(const float* A2, const float* w3, const float* b3, int64_t n,
                          const float* t, float* y, float* dy, double* sq) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  float acc = A2[row * kHid + lane] * w3[lane] + A2[row * kHid + lane + 64] * w3[lane + 64];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    const float out = acc + b3[0];
    y[row] = out;
    if (t) {
      const float r = out - t[row];
      dy[row] = 2.0f * r / (float)n;
      sq[row] = (double)r * (double)r;
    }
  }
}

// dZ2[b][j] = dy[b] w3[j] gelu'(Z2[b][j])
__global__ void k_mlp_dz2(const float* Z2, const float* dy, const float* w3, int64_t n, float* dZ2) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * kHid) return;
  const int64_t b = idx / kHid, j = idx - b * kHid;
  dZ2[idx] = dy[b] * w3[j] * gelu_grad(Z2[idx]);
}

// Column sums of a [n][cols] matrix (rows optionally weighted by wrow[b]),
// first stage: workgroup g sums rows [g*R, (g+1)*R) into part[g][col]
// (double).  cols <= 256; thread c handles column c.
__global__ void k_col_partial(const float* A, const float* wrow, int64_t n, int64_t cols,
                              int64_t R, double* part) {
  const int64_t g = blockIdx.x;
  const int c = threadIdx.x;
  if (c >= cols) return;
  const int64_t r0 = g * R, r1 = (r0 + R) < n ? (r0 + R) : n;
  double s = 0.0;
  for (int64_t b = r0; b < r1; ++b) {
    const double a = A ? (double)A[b * cols + c] : 1.0;
    s += wrow ? a * (double)wrow[b] : a;
  }
  part[g * cols + c] = s;
}

// out[i] (float) = sum_z part[z][i] (fixed order)
__global__ void k_sum_parts(const double* part, int64_t nz, int64_t len, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = 0.0;
  for (int64_t z = 0; z < nz; ++z) s += part[z * len + i];
  out[i] = (float)s;
}

// loss = sum sq / n (one workgroup, fixed order)
__global__ void k_loss(const double* sq, int64_t n, double* loss) {
  double v[1] = {0.0};
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) v[0] += sq[i];
  block_sum<1>(v);
  if (threadIdx.x == 0) *loss = v[0] / (double)n;
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction for step t >= 1.
__global__ void k_adam(float* p, float* m, float* v, const float* g, int64_t len, float lr,
                       float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// BF16 inference of the whole network, one workgroup (4 waves) per 64 rows,
// 16 rows per wave.  Every matrix operand is rounded to BF16 (nearest even):
// X, W1, the first hidden activations, W2, the second hidden activations and
// w3; products on v_mfma_f32_16x16x32_bf16 (layer 1's k = 16 padded to 32
// with zeros) with FP32 accumulation; biases and GELU in FP32; the output
// layer is an FP32 dot product of the BF16 values.  Fragments: lane l holds
// k = 8 (l / 16) .. + 7 of row l % 16 (A) or column l % 16 (B); accumulator
// element q of lane l is row 4 (l / 16) + q, column l % 16.
constexpr int kBfPitch = kHid + 8;  // LDS row pitch (272 bytes: 16-byte aligned rows)
__global__ __launch_bounds__(256) void k_mlp_forward_bf16(const float* __restrict__ P, int64_t n,
                                                          const float* __restrict__ X,
                                                          float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) __bf16 W2s[kHid * kBfPitch];
  __shared__ __attribute__((aligned(16))) __bf16 W1s[kHid * 40];
  __shared__ __attribute__((aligned(16))) __bf16 Hs[4][16 * kBfPitch];
  __shared__ float w3s[kHid];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kHid * kHid; e += 256)
    W2s[(e / kHid) * kBfPitch + (e % kHid)] = (__bf16)P[kOffW2 + e];
  for (int e = tid; e < kHid * 32; e += 256) {
    const int j = e / 32, k = e % 32;
    W1s[j * 40 + k] = k < kIn ? (__bf16)P[kOffW1 + j * kIn + k] : (__bf16)0.0f;
  }
  if (tid < kHid) w3s[tid] = (float)(__bf16)P[kOffW3 + tid];
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int rl = lane & 15, kg = lane >> 4;
  // layer 1: A = X rows (k 0..15, zeros beyond)
  bf16x8 a;
  {
    const int64_t row = r0 + rl;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * kg + j;
      a[j] = (row < n && k < kIn) ? (__bf16)X[row * kIn + k] : (__bf16)0.0f;
    }
  }
  __bf16* H = Hs[wave];
#pragma unroll
  for (int jt = 0; jt < kHid / 16; ++jt) {
    const int col = jt * 16 + rl;
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(&W1s[col * 40 + 8 * kg]);
    f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    const float bias = P[kOffB1 + col];
#pragma unroll
    for (int q = 0; q < 4; ++q) H[(4 * kg + q) * kBfPitch + col] = (__bf16)gelu(acc[q] + bias);
  }
  __syncthreads();
  // layer 2 and the output layer
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int jt = 0; jt < kHid / 16; ++jt) {
    const int col = jt * 16 + rl;
    f32x4 acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kHid / 32; ++ks) {
      const bf16x8 ha = *reinterpret_cast<const bf16x8*>(&H[rl * kBfPitch + ks * 32 + 8 * kg]);
      const bf16x8 wb = *reinterpret_cast<const bf16x8*>(&W2s[col * kBfPitch + ks * 32 + 8 * kg]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha, wb, acc, 0, 0, 0);
    }
    const float bias = P[kOffB2 + col];
#pragma unroll
    for (int q = 0; q < 4; ++q) part[q] += (float)(__bf16)gelu(acc[q] + bias) * w3s[col];
  }
  // sum over the 16 lanes of a row group (the columns), fixed pattern
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) part[q] += __shfl_xor(part[q], off, 64);
  if (rl == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = r0 + 4 * kg + q;
      if (row < n) y[row] = part[q] + P[kOffB3];
    }
  }
}

// Per-state features of the first iteration (see qsgw.h), standardized as
// (f - mean) / scale when mean is given.
__global__ void k_mlp_features(int64_t nbf, int64_t nocc, const double* eps, const double* diag,
                               const float* mean, const float* scale, float* X) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nbf) return;
  const double e = eps[m], homo = eps[nocc - 1], lumo = eps[nocc];
  const double re = diag[m * 4 + 0], im = diag[m * 4 + 1], der = diag[m * 4 + 2],
               sx = diag[m * 4 + 3];
  const double z = 1.0 / (1.0 - der);
  double f[kIn];
  f[0] = e;
  f[1] = sx;
  f[2] = re;
  f[3] = der;
  f[4] = (double)nocc / (double)nbf;
  f[5] = lumo - homo;
  f[6] = im;
  f[7] = z;
  f[8] = m < nocc ? 1.0 : 0.0;
  f[9] = e - homo;
  f[10] = e - lumo;
  f[11] = (double)nbf / 120.0;
  f[12] = (double)m / (double)nbf;
  f[13] = z * re;
  f[14] = fabs(der) > 1.0 ? 1.0 : 0.0;
  f[15] = 1.0;
#pragma unroll
  for (int q = 0; q < kIn; ++q) {
    float x = (float)f[q];
    if (mean) x = (x - mean[q]) / scale[q];
    X[m * kIn + q] = x;
  }
}

// Warm start: e'_m = eps0_m + delta_m, stably sorted; perm[r] = state of rank r.
__global__ void k_warm_rank(int64_t nbf, const double* eps0, const float* delta, double* eps,
                            int64_t* perm) {
  for (int64_t m = threadIdx.x; m < nbf; m += blockDim.x) {
    const double em = eps0[m] + (double)delta[m];
    int64_t r = 0;
    for (int64_t j = 0; j < nbf; ++j) {
      const double ej = eps0[j] + (double)delta[j];
      r += (ej < em || (ej == em && j < m)) ? 1 : 0;
    }
    eps[r] = em;
    perm[r] = m;
  }
}

// C[:, r] = C0[:, perm[r]]
__global__ void k_warm_permute(int64_t nbf, const double* C0, const int64_t* perm, double* C) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbf * nbf) return;
  const int64_t row = idx / nbf, r = idx - row * nbf;
  C[idx] = C0[row * nbf + perm[r]];
}

struct MlpBuffers {
  float *Z1, *A1, *Z2, *A2, *dZ2, *dZ1, *y, *dy, *grad;
  double *sq, *part, *cpart;
};

int mlp_buffers(qsgw_ctx* c, int64_t n, int64_t nz, int64_t ngroups, MlpBuffers* b) {
  float* f = nullptr;
  double* d = nullptr;
  const size_t nf = (size_t)(6 * n * kHid + 2 * n + kNParams + 64);
  const size_t ndd = (size_t)(n + nz * (kHid * kHid + kHid * kIn) + ngroups * (3 * kHid + 2) + 64);
  CHECK(ws_get(c, W_MLP_F32, nf, &f));
  CHECK(ws_get(c, W_MLP_F64, ndd, &d));
  b->Z1 = f;
  b->A1 = b->Z1 + n * kHid;
  b->Z2 = b->A1 + n * kHid;
  b->A2 = b->Z2 + n * kHid;
  b->dZ2 = b->A2 + n * kHid;
  b->dZ1 = b->dZ2 + n * kHid;
  b->y = b->dZ1 + n * kHid;
  b->dy = b->y + n;
  b->grad = b->dy + n;
  b->sq = d;
  b->part = b->sq + n;
  b->cpart = b->part + nz * (kHid * kHid + kHid * kIn);
  return QSGW_OK;
}

// Forward through both hidden layers into the buffers.
int mlp_hidden(qsgw_ctx* c, const float* P, int64_t n, const float* X, MlpBuffers& b, bool keepZ) {
  CHECK((gemm_t<float, 64, 64, false>(
      c, "mlp layer 1", Strided<true, float>{X, kIn, 1, 0, n},
      Strided<true, float>{P + kOffW1, kIn, 1, 0, kHid},
      EpiBiasGelu{P + kOffB1, keepZ ? b.Z1 : nullptr, b.A1, kHid}, n, kHid, kIn, 1)));
  CHECK((gemm_t<float, 64, 64, false>(
      c, "mlp layer 2", Strided<true, float>{b.A1, kHid, 1, 0, n},
      Strided<true, float>{P + kOffW2, kHid, 1, 0, kHid},
      EpiBiasGelu{P + kOffB2, keepZ ? b.Z2 : nullptr, b.A2, kHid}, n, kHid, kHid, 1)));
  return QSGW_OK;
}

int check_n(qsgw_ctx* c, int64_t n) {
  if (n < 1 || n > (1LL << 26)) return fail(c, QSGW_ERR_INVALID_ARG, "need 1 <= n <= 2^26 states");
  return QSGW_OK;
}

}  // namespace

extern "C" {

int qsgw_mlp_forward(qsgw_ctx* c, const float* params, int64_t n, const float* X, float* y) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  CHECK(check_n(c, n));
  if (!params || !X || !y) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  CHECK(check_finite(c, "qsgw_mlp_forward",
                     {fin32(params, kNParams, "params"), fin32(X, n * kIn, "X")}));
  MlpBuffers b;
  CHECK(mlp_buffers(c, n, 1, 1, &b));
  CHECK(mlp_hidden(c, params, n, X, b, false));
  hipLaunchKernelGGL(k_mlp_out, dim3(blocks_for(n, 4)), dim3(256), 0, c->stream, b.A2,
                     params + kOffW3, params + kOffB3, n, (const float*)nullptr, y, (float*)nullptr,
                     (double*)nullptr);
  return launch_check(c, "k_mlp_out");
}

int qsgw_mlp_forward_bf16(qsgw_ctx* c, const float* params, int64_t n, const float* X, float* y) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  CHECK(check_n(c, n));
  if (!params || !X || !y) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  CHECK(check_finite(c, "qsgw_mlp_forward_bf16",
                     {fin32(params, kNParams, "params"), fin32(X, n * kIn, "X")}));
  hipLaunchKernelGGL(k_mlp_forward_bf16, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, c->stream,
                     params, n, X, y);
  return launch_check(c, "k_mlp_forward_bf16");
}

int qsgw_mlp_train_step(qsgw_ctx* c, float* params, float* adam_m, float* adam_v, int64_t step,
                        double lr, int64_t n, const float* X, const float* target, float* grad,
                        double* loss) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  CHECK(check_n(c, n));
  if (!params || !adam_m || !adam_v || !X || !target)
    return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  if (step < 1) return fail(c, QSGW_ERR_INVALID_ARG, "Adam steps count from 1");
  if (!(lr >= 0.0) || !isfinite(lr)) return fail(c, QSGW_ERR_INVALID_ARG, "need a finite lr >= 0");
  CHECK(check_finite(c, "qsgw_mlp_train_step",
                     {fin32(params, kNParams, "params"), fin32(adam_m, kNParams, "adam_m"),
                      fin32(adam_v, kNParams, "adam_v"), fin32(X, n * kIn, "X"),
                      fin32(target, n, "target")}));
  // weight gradients reduce over the batch: split K = n in chunks of 512
  const SplitPlan sp = split_plan(n, (n + 511) / 512);
  const int64_t R = 1024, ngroups = (n + R - 1) / R;
  MlpBuffers b;
  CHECK(mlp_buffers(c, n, sp.nz, ngroups, &b));
  CHECK(mlp_hidden(c, params, n, X, b, true));
  hipLaunchKernelGGL(k_mlp_out, dim3(blocks_for(n, 4)), dim3(256), 0, c->stream, b.A2,
                     params + kOffW3, params + kOffB3, n, target, b.y, b.dy, b.sq);
  CHECK(launch_check(c, "k_mlp_out"));
  hipLaunchKernelGGL(k_mlp_dz2, dim3(blocks_for(n * kHid)), dim3(256), 0, c->stream, b.Z2, b.dy,
                     params + kOffW3, n, b.dZ2);
  CHECK(launch_check(c, "k_mlp_dz2"));
  float* g = grad ? grad : b.grad;
  // output layer: dw3 = A2^T dy, db3 = sum dy
  double* cp = b.cpart;
  hipLaunchKernelGGL(k_col_partial, dim3((unsigned)ngroups), dim3(256), 0, c->stream, b.A2, b.dy, n,
                     (int64_t)kHid, R, cp);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c->stream, cp, ngroups, (int64_t)kHid,
                     g + kOffW3);
  cp += ngroups * kHid;
  hipLaunchKernelGGL(k_col_partial, dim3((unsigned)ngroups), dim3(256), 0, c->stream,
                     (const float*)nullptr, b.dy, n, (int64_t)1, R, cp);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c->stream, cp, ngroups, (int64_t)1,
                     g + kOffB3);
  cp += ngroups;
  // layer 2: dW2[i][j] = sum_b dZ2[b][i] A1[b][j], db2 = colsum dZ2
  CHECK((gemm_t<float, 64, 64, false>(
      c, "mlp dW2", Strided<false, float>{b.dZ2, 1, kHid, 0, kHid},
      Strided<false, float>{b.A1, 1, kHid, 0, kHid},
      EpiStore{b.part, kHid, 0, kHid * kHid, 1.0}, kHid, kHid, n, 1, sp)));
  hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(kHid * kHid)), dim3(256), 0, c->stream, b.part,
                     sp.nz, (int64_t)(kHid * kHid), g + kOffW2);
  hipLaunchKernelGGL(k_col_partial, dim3((unsigned)ngroups), dim3(256), 0, c->stream, b.dZ2,
                     (const float*)nullptr, n, (int64_t)kHid, R, cp);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c->stream, cp, ngroups, (int64_t)kHid,
                     g + kOffB2);
  cp += ngroups * kHid;
  // dZ1 = (dZ2 W2) * gelu'(Z1)
  CHECK((gemm_t<float, 64, 64, false>(
      c, "mlp dA1", Strided<true, float>{b.dZ2, kHid, 1, 0, n},
      Strided<false, float>{params + kOffW2, 1, kHid, 0, kHid}, EpiGeluGrad{b.Z1, b.dZ1, kHid}, n,
      kHid, kHid, 1)));
  // layer 1: dW1[i][q] = sum_b dZ1[b][i] X[b][q], db1 = colsum dZ1
  CHECK((gemm_t<float, 64, 64, false>(
      c, "mlp dW1", Strided<false, float>{b.dZ1, 1, kHid, 0, kHid},
      Strided<false, float>{X, 1, kIn, 0, kIn}, EpiStore{b.part, kIn, 0, kHid * kIn, 1.0}, kHid,
      kIn, n, 1, sp)));
  hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(kHid * kIn)), dim3(256), 0, c->stream, b.part,
                     sp.nz, (int64_t)(kHid * kIn), g + kOffW1);
  hipLaunchKernelGGL(k_col_partial, dim3((unsigned)ngroups), dim3(256), 0, c->stream, b.dZ1,
                     (const float*)nullptr, n, (int64_t)kHid, R, cp);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c->stream, cp, ngroups, (int64_t)kHid,
                     g + kOffB1);
  CHECK(launch_check(c, "mlp gradient"));
  if (loss) {
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, c->stream, b.sq, n, loss);
    CHECK(launch_check(c, "k_loss"));
  }
  const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(kNParams)), dim3(256), 0, c->stream, params, adam_m,
                     adam_v, g, kNParams, (float)lr, c1, c2);
  return launch_check(c, "k_adam");
}

int qsgw_mlp_features(qsgw_ctx* c, int64_t nbf, int64_t nocc, const double* eps, const double* diag,
                      const float* mean, const float* scale, float* X) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  if (!eps || !diag || !X || (!mean) != (!scale))
    return fail(c, QSGW_ERR_INVALID_ARG, "null pointer (mean and scale go together)");
  CHECK(check_finite(c, "qsgw_mlp_features",
                     {fin(eps, nbf, "eps"), fin(diag, 4 * nbf, "diag"), fin32(mean, kIn, "mean"),
                      fin32(scale, kIn, "scale")}));
  hipLaunchKernelGGL(k_mlp_features, dim3(blocks_for(nbf)), dim3(256), 0, c->stream, nbf, nocc, eps,
                     diag, mean, scale, X);
  return launch_check(c, "k_mlp_features");
}

int qsgw_warm_start(qsgw_ctx* c, int64_t nbf, const double* eps0, const double* C0,
                    const float* delta, double* eps, double* C) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (nbf < 1 || nbf > 46340) return fail(c, QSGW_ERR_INVALID_ARG, "bad nbf");
  if (!eps0 || !C0 || !delta || !eps || !C) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  if (eps == eps0 || C == C0) return fail(c, QSGW_ERR_INVALID_ARG, "outputs must not alias inputs");
  CHECK(check_finite(c, "qsgw_warm_start", {fin(eps0, nbf, "eps0"), fin(C0, nbf * nbf, "C0"),
                                            fin32(delta, nbf, "delta")}));
  int64_t* perm = nullptr;
  CHECK(ws_get(c, W_MLP_PERM, (size_t)nbf, &perm));
  hipLaunchKernelGGL(k_warm_rank, dim3(1), dim3(1024), 0, c->stream, nbf, eps0, delta, eps, perm);
  hipLaunchKernelGGL(k_warm_permute, dim3(blocks_for(nbf * nbf)), dim3(256), 0, c->stream, nbf, C0,
                     perm, C);
  return launch_check(c, "warm start");
}

}  // extern "C"
