// Plain kernels of the qsGW iteration (see kernels.hpp for the contracts).
#include "kernels.hpp"

#include <math.h>

namespace qsgw {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

}  // namespace

__global__ void k_transitions(const double* eps, int64_t nocc, int64_t nv, double* delta,
                              double* sqrt_delta, int* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nocc * nv) return;
  const int64_t i = t / nv;
  const int64_t a = nocc + (t - i * nv);
  const double d = eps[a] - eps[i];
  if (!(d > 0.0) || !finite(d)) atomicOr(bad, 1);
  delta[t] = d;
  sqrt_delta[t] = sqrt(d > 0.0 ? d : 0.0);
}

__global__ void k_gather_bia(const double* bmo, const double* sqrt_delta, int64_t naux,
                             int64_t nbf, int64_t nocc, double* bt, float* bt32) {
  const int64_t nv = nbf - nocc;
  const int64_t ntr = nocc * nv;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= naux * ntr) return;
  const int64_t P = idx / ntr;
  const int64_t t = idx - P * ntr;
  const int64_t i = t / nv;
  const int64_t a = nocc + (t - i * nv);
  const double v = bmo[(P * nbf + i) * nbf + a] * (sqrt_delta ? sqrt_delta[t] : 1.0);
  bt[idx] = v;
  if (bt32) bt32[idx] = (float)v;
}

__global__ void k_omega_from_eigs(const double* lam, int64_t n, double* Omega, int* bad) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double l = lam[s];
  if (!(l > 0.0) || !finite(l)) atomicOr(bad, 1);
  Omega[s] = sqrt(l > 0.0 ? l : 0.0);
}

__global__ void k_reduce_sym(const double* part, int64_t nz, int64_t n, double* out,
                             int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t m = idx / n;
  const int64_t c = idx - m * n;
  const int64_t nn = n * n;
  double a = 0.0, b = 0.0;
  for (int64_t z = 0; z < nz; ++z) {
    a += part[z * nn + m * n + c];
    b += part[z * nn + c * n + m];
  }
  // a + b and b + a round identically, so out stays exactly symmetric.
  const double v = 0.5 * (a + b);
  out[idx] = accumulate ? out[idx] + v : v;
}

__global__ void k_sum_slices(const double* part, int64_t nz, int64_t len, int64_t zg,
                             double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ng = (nz + zg - 1) / zg;
  if (idx >= ng * len) return;
  const int64_t g = idx / len, e = idx - g * len;
  const int64_t z1 = (g + 1) * zg < nz ? (g + 1) * zg : nz;
  double a = 0.0;
  for (int64_t z = g * zg; z < z1; ++z) a += part[z * len + e];
  out[idx] = a;
}

__global__ void k_rho_reduce(const double* part, int64_t nz, int64_t rows, int64_t ns,
                             const double* Omega, double* rho, float* rho32) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t len = rows * ns;
  if (idx >= len) return;
  double v = 0.0;
  for (int64_t z = 0; z < nz; ++z) v += part[z * len + idx];
  const double r = v * sqrt(2.0 / Omega[idx % ns]);
  rho[idx] = r;
  if (rho32) rho32[idx] = (float)r;
}

__global__ void k_to_f32(const double* in, int64_t n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// One thread per chunk (row, k-block): 8 FP64 values rounded to FP32 and
// split into hi and lo BF16 halves (x = hi + lo to 16 significant bits).
__device__ __forceinline__ void split_chunk(const double (&x)[8], uint16_t* hi, uint16_t* lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) split_bf16x2((float)x[2 * u], (float)x[2 * u + 1], h[u], l[u]);
  *reinterpret_cast<uint4*>(hi) = uint4{h[0], h[1], h[2], h[3]};
  *reinterpret_cast<uint4*>(lo) = uint4{l[0], l[1], l[2], l[3]};
}

__global__ void k_split_pairs(const double* bmo, const int32_t* blocks, int64_t nblk, int64_t nbf,
                              int64_t naux, int64_t kpad, uint16_t* out) {
  const int64_t rows = nblk * 128, nkb = kpad / 8;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * nkb) return;
  const int64_t r = idx % rows, kb = idx / rows;
  int64_t m, k;
  pair_of<8, 16>(blocks, r >> 7, (int)(r & 127), m, k);
  const bool ok = m < nbf && k < nbf;
  const int64_t nn = nbf * nbf;
  double x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t P = kb * 8 + j;
    x[j] = (ok && P < naux) ? bmo[P * nn + m * nbf + k] : 0.0;
  }
  const int64_t o = (kb * rows + r) * 8;
  split_chunk(x, out + o, out + nkb * rows * 8 + o);
}

__global__ void k_zero_u16(uint16_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_split_rows(const double* in, int64_t ld, int64_t rows, int64_t K,
                             int64_t rows_pad, int64_t kpad, uint16_t* out) {
  // 32 rows x 256 k per workgroup through LDS: rows are read along k
  // (coalesced), chunks are written along r (adjacent rows adjacent).
  constexpr int TR = 32, TK = 256, PITCH = TK + 4;
  __shared__ __attribute__((aligned(16))) float t[TR * PITCH];
  const int64_t r0 = (int64_t)blockIdx.x * TR, k0 = (int64_t)blockIdx.y * TK;
  const int tid = threadIdx.x;
  for (int rr = 0; rr < TR; ++rr) {
    const int64_t r = r0 + rr, k = k0 + tid;
    t[rr * PITCH + tid] = (r < rows && k < K) ? (float)in[r * ld + k] : 0.0f;
  }
  __syncthreads();
  const int64_t nkb = kpad / 8;
  for (int q = tid; q < TR * (TK / 8); q += blockDim.x) {
    const int rr = q % TR, kbl = q / TR;
    const int64_t kb = k0 / 8 + kbl;
    if (kb >= nkb) continue;
    const float* x = t + rr * PITCH + 8 * kbl;
    uint32_t h[4], l[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) split_bf16x2(x[2 * u], x[2 * u + 1], h[u], l[u]);
    const int64_t o = (kb * rows_pad + r0 + rr) * 8;
    *reinterpret_cast<uint4*>(out + o) = uint4{h[0], h[1], h[2], h[3]};
    *reinterpret_cast<uint4*>(out + nkb * rows_pad * 8 + o) = uint4{l[0], l[1], l[2], l[3]};
  }
}

__global__ void k_split_cols(const double* in, int64_t ld, int64_t rows, int64_t K,
                             int64_t rows_pad, int64_t kpad, uint16_t* out) {
  const int64_t nkb = kpad / 8;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows_pad * nkb) return;
  const int64_t r = idx % rows_pad, kb = idx / rows_pad;
  double x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t k = kb * 8 + j;
    x[j] = (r < rows && k < K) ? in[k * ld + r] : 0.0;
  }
  const int64_t o = (kb * rows_pad + r) * 8;
  split_chunk(x, out + o, out + nkb * rows_pad * 8 + o);
}

__global__ void k_occ_trace(const double* bmo, int64_t naux, int64_t nbf, int64_t nocc,
                            double* c) {
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= naux) return;
  double s = 0.0;
  for (int64_t i = 0; i < nocc; ++i) s += bmo[(P * nbf + i) * nbf + i];
  c[P] = s;
}

__global__ void k_hartree_part(const double* bmo, const double* c, int64_t naux, int64_t nn,
                               int64_t pg, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ng = (naux + pg - 1) / pg;
  if (idx >= ng * nn) return;
  const int64_t g = idx / nn, e = idx - g * nn;
  const int64_t p1 = (g + 1) * pg < naux ? (g + 1) * pg : naux;
  double s = 0.0;
  for (int64_t P = g * pg; P < p1; ++P) s += c[P] * bmo[P * nn + e];
  out[idx] = 2.0 * s;
}

__global__ void k_fock_assemble(const double* hmo, const double* J, const double* Kpart,
                                int64_t nz, const double* V, int64_t n, double* F) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t m = idx / n;
  const int64_t c = idx - m * n;
  const int64_t nn = n * n;
  double k = 0.0;
  for (int64_t z = 0; z < nz; ++z) k += Kpart[z * nn + idx];
  const double h = 0.5 * (hmo[m * n + c] + hmo[c * n + m]);
  F[idx] = h + J[idx] - k + V[idx];
}

__global__ void k_hf_core_mo(const double* eps, const double* J, const double* Kpart, int64_t nz,
                             int64_t n, double* X) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t m = idx / n;
  const int64_t c = idx - m * n;
  const int64_t nn = n * n;
  double k = 0.0;
  for (int64_t z = 0; z < nz; ++z) k += Kpart[z * nn + idx];
  X[idx] = (m == c ? eps[m] : 0.0) - J[idx] + k;
}

__global__ void k_symmetrize(const double* a, int64_t n, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t m = idx / n;
  const int64_t c = idx - m * n;
  out[idx] = 0.5 * (a[m * n + c] + a[c * n + m]);
}

__global__ void k_axpby(const double* a, const double* b, double alpha, double beta, int64_t len,
                        double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= len) return;
  out[idx] = alpha * a[idx] + beta * b[idx];
}

// One workgroup (256 threads) per column j: the first row of largest |C[r][j]|
// decides the sign (larger magnitude wins, ties go to the smaller row).
__global__ void k_fix_column_signs(double* C, int64_t n) {
  __shared__ double sm[256];
  __shared__ int64_t sr[256];
  const int64_t j = blockIdx.x;
  if (j >= n) return;
  double best = -1.0;
  int64_t br = n;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double a = fabs(C[r * n + j]);
    if (a > best) {  // rows ascend per thread: the first maximum is kept
      best = a;
      br = r;
    }
  }
  sm[threadIdx.x] = best;
  sr[threadIdx.x] = br;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = sm[threadIdx.x + w];
      const int64_t orow = sr[threadIdx.x + w];
      if (o > sm[threadIdx.x] || (o == sm[threadIdx.x] && orow < sr[threadIdx.x])) {
        sm[threadIdx.x] = o;
        sr[threadIdx.x] = orow;
      }
    }
    __syncthreads();
  }
  const bool flip = sr[0] < n && C[sr[0] * n + j] < 0.0;
  __syncthreads();
  if (flip)
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) C[r * n + j] = -C[r * n + j];
}

__global__ void k_max_abs_diff(const double* a, const double* b, int64_t n, double* out) {
  __shared__ double red[4];
  double m = 0.0;
  bool nonfinite = false;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = fabs(a[i] - b[i]);
    if (!finite(d)) nonfinite = true;
    m = fmax(m, d);
  }
  if (nonfinite) m = INFINITY;
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    *out = r;
  }
}

__global__ void k_diis_error_mo(const double* F, int64_t n, int64_t nocc, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t m = idx / n, k = idx - m * n;
  const double om = m < nocc ? 1.0 : 0.0, ok = k < nocc ? 1.0 : 0.0;
  out[idx] = F[idx] * (ok - om);
}

__global__ void k_diis_dots(const double* E, int64_t len, int64_t k, const int* slots, double* B,
                            int64_t ld) {
  __shared__ double red[4];
  const int64_t j = slots[blockIdx.x];
  const double* a = E + k * len;
  const double* b = E + j * len;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += blockDim.x) s += a[i] * b[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    B[k * ld + j] = t;
    B[j * ld + k] = t;
  }
}

__global__ void k_diis_solve(const double* B, int64_t ld, const int* slots, int nact, double* c,
                             int* bad) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  constexpr int kMax = 17;
  double a[kMax][kMax + 1];
  const int n = nact + 1;
  for (int i = 0; i < nact; ++i) {
    for (int j = 0; j < nact; ++j) a[i][j] = B[(int64_t)slots[i] * ld + slots[j]];
    a[i][nact] = -1.0;
    a[i][n] = 0.0;
  }
  for (int j = 0; j < nact; ++j) a[nact][j] = -1.0;
  a[nact][nact] = 0.0;
  a[nact][n] = -1.0;
  bool singular = false;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (a[piv][col] == 0.0) {
      singular = true;
      break;
    }
    if (piv != col)
      for (int q = col; q <= n; ++q) {
        const double t = a[col][q];
        a[col][q] = a[piv][q];
        a[piv][q] = t;
      }
    for (int r = col + 1; r < n; ++r) {
      const double f = a[r][col] / a[col][col];
      for (int q = col; q <= n; ++q) a[r][q] -= f * a[col][q];
    }
  }
  double x[kMax];
  if (!singular) {
    for (int r = n - 1; r >= 0; --r) {
      double t = a[r][n];
      for (int q = r + 1; q < n; ++q) t -= a[r][q] * x[q];
      x[r] = t / a[r][r];
    }
    for (int i = 0; i < nact; ++i)
      if (!isfinite(x[i])) singular = true;
  }
  if (singular) {
    *bad = 1;
    for (int i = 0; i < nact; ++i) c[i] = i == nact - 1 ? 1.0 : 0.0;
  } else {
    for (int i = 0; i < nact; ++i) c[i] = x[i];
  }
}

__global__ void k_diis_combine(const double* F, int64_t len, const int* slots, int nact,
                               const double* c, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int i = 0; i < nact; ++i) s += c[i] * F[(int64_t)slots[i] * len + e];
  out[e] = s;
}

template <class T>
__device__ __forceinline__ void check_finite_body(const T* x, int64_t len, int* bad, int mask) {
  bool ok = true;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    ok = ok && isfinite(x[i]);
  if (!ok) atomicOr(bad, mask);
}
__global__ void k_scale_rho(double* rho, int64_t naux, int64_t ntr, const double* Omega) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= naux * ntr) return;
  rho[idx] *= sqrt(2.0 / Omega[idx % ntr]);
}

__global__ void k_check_finite(const double* x, int64_t len, int* bad, int mask) {
  check_finite_body(x, len, bad, mask);
}
__global__ void k_check_finite_f32(const float* x, int64_t len, int* bad, int mask) {
  check_finite_body(x, len, bad, mask);
}

// Order-independent fingerprint of an array's bit patterns:
// sum_i bits(x_i) * (2 i + 1) mod 2^64.  Integer sums wrap and commute, so
// the result does not depend on the reduction order.
__global__ void k_bits_fingerprint(const double* x, int64_t len, unsigned long long* out) {
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += (unsigned long long)__double_as_longlong(x[i]) * (unsigned long long)(2 * i + 1);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

// Fock matrix with a frozen mean field, MO basis: F = (hmo + hmo^T) / 2 + V.
__global__ void k_fock_frozen(const double* hmo, const double* V, int64_t n, double* F) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t m = idx / n;
  const int64_t c = idx - m * n;
  F[idx] = 0.5 * (hmo[m * n + c] + hmo[c * n + m]) + V[idx];
}

// One workgroup per (state, block of OT frequencies).  Threads stride over the
// (k, s) pairs of w[m][k][s] (unit stride in s), accumulate OT complex pole
// sums in registers, then reduce in a fixed order (wave shuffles, then the 4
// waves in index order): the result is deterministic.
__global__ void k_sigma_diag_grid(const double* w, const double* eps, const double* Omega,
                                  int64_t nbf, int64_t nocc, int64_t ns, double eta,
                                  const double* omega, int64_t nomega, const int64_t* states,
                                  int64_t nstates, double* out, int accumulate, int* bad) {
  constexpr int OT = 8;
  __shared__ double red[4][2 * OT];
  const int64_t j = blockIdx.x;
  const int64_t l0 = (int64_t)blockIdx.y * OT;
  if (j >= nstates) return;
  const int64_t m = states[j];
  if (m < 0 || m >= nbf) {
    if (threadIdx.x == 0) atomicOr(bad, 1);
    return;
  }
  double om[OT];
#pragma unroll
  for (int q = 0; q < OT; ++q) om[q] = (l0 + q < nomega) ? omega[l0 + q] : 0.0;
  double re[OT], im[OT];
#pragma unroll
  for (int q = 0; q < OT; ++q) re[q] = im[q] = 0.0;
  const double eta2 = eta * eta;
  const int64_t npair = nbf * ns;
  const double* wm = w + m * npair;
  for (int64_t p = threadIdx.x; p < npair; p += blockDim.x) {
    const int64_t k = p / ns;
    const int64_t s = p - k * ns;
    const double x = wm[p];
    const double w2 = x * x;
    const bool occ = k < nocc;
    const double shift = occ ? (Omega[s] - eps[k]) : (-Omega[s] - eps[k]);
    const double sg = occ ? eta : -eta;
#pragma unroll
    for (int q = 0; q < OT; ++q) {
      const double d = om[q] + shift;
      const double inv = w2 / (d * d + eta2);
      re[q] += d * inv;
      im[q] += sg * inv;
    }
  }
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < OT; ++q) {
    const double a = wave_sum(re[q]);
    const double b = wave_sum(im[q]);
    if ((threadIdx.x & 63) == 0) {
      red[wv][2 * q] = a;
      red[wv][2 * q + 1] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * OT) {
    const int q = threadIdx.x >> 1;
    double v = 0.0;
    for (int u = 0; u < (int)(blockDim.x >> 6); ++u) v += red[u][threadIdx.x];
    const int64_t l = l0 + q;
    if (l < nomega) {
      double* o = out + (j * nomega + l) * 2 + (threadIdx.x & 1);
      *o = accumulate ? *o + v : v;
    }
  }
}

__global__ void k_sigma_diag_self(const double* w, const double* eps, const double* Omega,
                                  int64_t nbf, int64_t nocc, int64_t ns, double eta,
                                  const int64_t* states, int64_t nstates, double* out, int64_t ld,
                                  int accumulate, int* bad) {
  const int64_t j = blockIdx.x;
  if (j >= nstates) return;
  const int64_t m = states ? states[j] : j;
  if (m < 0 || m >= nbf) {
    if (threadIdx.x == 0) atomicOr(bad, 1);
    return;
  }
  double r[3] = {0.0, 0.0, 0.0};
  diag_self_partial(w + m * nbf * ns, eps, Omega, m, nbf, nocc, ns, eta, r);
  block_sum<3>(r);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) out[j * ld + q] = accumulate ? out[j * ld + q] + r[q] : r[q];
}

__global__ void k_exchange_diag(const double* bmo, int64_t naux, int64_t nbf, int64_t nocc,
                                double* out, int64_t ld) {
  const int64_t m = blockIdx.x;
  if (m >= nbf) return;
  double v[1] = {exchange_diag_partial(bmo, naux, nbf, nocc, m)};
  block_sum<1>(v);
  if (threadIdx.x == 0) out[m * ld] = v[0];
}

namespace {
// first index s in [0, n) with a[s] > x (a ascending), n if none
__device__ __forceinline__ int64_t first_above(const double* a, int64_t n, double x) {
  int64_t l = 0, h = n;
  while (l < h) {
    const int64_t mid = (l + h) >> 1;
    if (a[mid] > x) h = mid; else l = mid + 1;
  }
  return l;
}
// first index s with a[s] >= x
__device__ __forceinline__ int64_t first_at_least(const double* a, int64_t n, double x) {
  int64_t l = 0, h = n;
  while (l < h) {
    const int64_t mid = (l + h) >> 1;
    if (a[mid] >= x) h = mid; else l = mid + 1;
  }
  return l;
}
}  // namespace

__global__ void k_near_ranges(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                              int64_t ns, double thr, int64_t ntiles, int64_t* lo, int64_t* cnt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntiles * nbf) return;
  const int64_t t = idx / nbf, k = idx - t * nbf;
  const int64_t m0 = t * 64, m1 = (m0 + 64 < nbf ? m0 + 64 : nbf) - 1;
  const double elo = eps[m0], ehi = eps[m1], ek = eps[k];
  // occupied k: |eps_m - eps_k + Omega| < thr  <=>  Omega in (eps_k - eps_m - thr, eps_k - eps_m + thr)
  // empty k:    |eps_m - eps_k - Omega| < thr  <=>  Omega in (eps_m - eps_k - thr, eps_m - eps_k + thr)
  double a, b;
  if (k < nocc) {
    a = ek - ehi - thr;
    b = ek - elo + thr;
  } else {
    a = elo - ek - thr;
    b = ehi - ek + thr;
  }
  const double slack = 1e-12 * (1.0 + fabs(a) + fabs(b));
  const int64_t s0 = first_at_least(Omega, ns, a - slack);
  const int64_t s1 = first_above(Omega, ns, b + slack);
  lo[idx] = s0;
  cnt[idx] = s1 > s0 ? s1 - s0 : 0;
}

// x of the pole term (m, k, s), formed exactly as the residue epilogue forms it
__device__ __forceinline__ double pole_x(const double* eps, const double* Omega, int64_t nocc,
                                         int64_t m, int64_t k, int64_t s) {
  return (eps[m] - eps[k]) + (k < nocc ? 1.0 : -1.0) * Omega[s];
}

__global__ void k_near_colflags(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                                int64_t ns, int64_t nsp, double thr, int64_t* flag) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbf * nsp) return;
  const int64_t k = idx / nsp, s = idx - k * nsp;
  int64_t f = 0;
  if (s < ns) {
    // x = eps_m - c with c = eps_k -+ Omega_s: candidates m with eps_m near c
    const double c = eps[k] - (k < nocc ? 1.0 : -1.0) * Omega[s];
    const double slack = 1e-12 * (1.0 + fabs(c) + thr);
    const int64_t m0 = first_at_least(eps, nbf, c - thr - slack);
    const int64_t m1 = first_above(eps, nbf, c + thr + slack);
    for (int64_t m = m0; m < m1 && !f; ++m) f = fabs(pole_x(eps, Omega, nocc, m, k, s)) < thr;
  }
  flag[idx] = f;
}

__global__ void k_near_colidx(const int64_t* flag, const int64_t* off, const int64_t* base,
                              int64_t nbf, int64_t nsp, int32_t* colidx) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbf * nsp) return;
  colidx[idx] = flag[idx] ? (int32_t)(base[idx / nsp] + off[idx]) : -1;
}

__global__ void k_near_mk(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                          int64_t ns, int64_t nsp, double thr, const int32_t* colidx,
                          int32_t* c0, int32_t* slo, int32_t* len) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbf * nbf) return;
  const int64_t m = idx / nbf, k = idx - m * nbf;
  // |ea + sg Omega_s| < thr, ea = eps_m - eps_k: Omega_s in (-sg ea - thr, -sg ea + thr)
  const double ea = eps[m] - eps[k];
  const double ctr = k < nocc ? -ea : ea;
  const double slack = 1e-12 * (1.0 + fabs(ctr) + thr);
  int64_t a = first_at_least(Omega, ns, ctr - thr - slack);
  int64_t b = first_above(Omega, ns, ctr + thr + slack);
  while (a < b && !(fabs(pole_x(eps, Omega, nocc, m, k, a)) < thr)) ++a;
  while (b > a && !(fabs(pole_x(eps, Omega, nocc, m, k, b - 1)) < thr)) --b;
  len[idx] = (int32_t)(b - a);
  slo[idx] = (int32_t)a;
  c0[idx] = b > a ? colidx[k * nsp + a] : 0;
}

__global__ void k_near_product(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                               double eta, const int32_t* c0, const int32_t* slo,
                               const int32_t* len, const float* wN, int64_t kc, double* npart) {
  // The slice's terms are enumerated into LDS in batches (coefficient and
  // column), then every thread runs over the batch for its n: independent
  // coalesced loads, no per-term latency chain.
  constexpr int KCMAX = 64, BATCH = 1024, NJ = 8;  // nbf <= 256 NJ
  __shared__ int64_t start[KCMAX + 1];
  __shared__ double scoef[BATCH];
  __shared__ int32_t scol[BATCH];
  const int64_t m = blockIdx.x, z = blockIdx.y;
  const int64_t k0 = z * kc, k1 = (k0 + kc) < nbf ? (k0 + kc) : nbf;
  const int nk = (int)(k1 - k0);
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < nk; ++i) {
      start[i] = t;
      t += len[m * nbf + k0 + i];
    }
    start[nk] = t;
  }
  __syncthreads();
  const int64_t total = start[nk];
  double acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = 0.0;
  for (int64_t b0 = 0; b0 < total; b0 += BATCH) {
    const int64_t nb = (total - b0) < BATCH ? (total - b0) : BATCH;
    for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) {
      const int64_t t = b0 + q;
      int i = 0;
      while (start[i + 1] <= t) ++i;  // the k of term t
      const int64_t k = k0 + i, e = m * nbf + k, r = t - start[i];
      const int64_t c = c0[e] + r, sidx = slo[e] + r;
      const double x = pole_x(eps, Omega, nocc, m, k, sidx);
      scoef[q] = (double)wN[c * nbf + m] * (x / (x * x + eta * eta));
      scol[q] = (int32_t)c;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int64_t n = threadIdx.x + 256 * j;
      if (n < nbf) {
        double a = acc[j];
#pragma unroll 8
        for (int64_t q = 0; q < nb; ++q) a += scoef[q] * (double)wN[(int64_t)scol[q] * nbf + n];
        acc[j] = a;
      }
    }
    __syncthreads();
  }
  double* out = npart + (z * nbf + m) * nbf;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t n = threadIdx.x + 256 * j;
    if (n < nbf) out[n] = acc[j];
  }
}

__global__ void k_near_offsets(const int64_t* cnt, int64_t nbf, int64_t ntiles, int64_t* off,
                               int64_t* total, int64_t* base) {
  // one workgroup per tile: exclusive prefix over k in chunks of blockDim.x
  __shared__ int64_t sh[1024];
  __shared__ int64_t carry;
  const int64_t t = blockIdx.x;
  if (t >= ntiles) return;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t k0 = 0; k0 < nbf; k0 += blockDim.x) {
    const int64_t k = k0 + threadIdx.x;
    const int64_t v = k < nbf ? cnt[t * nbf + k] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (unsigned d = 1; d < blockDim.x; d <<= 1) {  // inclusive scan (Hillis-Steele)
      const int64_t add = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (k < nbf) off[t * nbf + k] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry += sh[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) total[t] = carry;
}

__global__ void k_near_bases(const int64_t* total, int64_t ntiles, int64_t* base) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t start = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    base[t] = start;
    start += total[t];
  }
}

__global__ void k_fill(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_near_fill(const int64_t* lo, const int64_t* cnt, const int64_t* off,
                            const int64_t* base, int64_t nbf, int64_t ntiles, int32_t* ktab,
                            int32_t* stab) {
  const int64_t idx = blockIdx.x;  // one workgroup per (tile, k)
  if (idx >= ntiles * nbf) return;
  const int64_t t = idx / nbf, k = idx - t * nbf;
  const int64_t n = cnt[idx], s0 = lo[idx], o = base[t] + off[idx];
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    ktab[o + j] = (int32_t)k;
    stab[o + j] = (int32_t)(s0 + j);
  }
}

// ------------------------------------------------------------------ qsMP2 --
// Right operand of the MP2 product for occupied p.  Element (n, p, ii, a') of
// the block: tb = ii nv + a', i = i0 + ii, a = nocc + a',
//   Rh[n][p][tb] = (2 (np|ia) - (pa|in)) x / (x^2 + eta^2),
//   x = eps_n + eps_a - eps_i - eps_p,
// with (np|ia) = D[n][p][tb] and (pa|in) = (ni|pa) read at
// xo + n xsn + i xsi + p nv + a'.
__global__ void k_mp2_rhs_occ(const double* D, const double* xo, int64_t xsn, int64_t xsi,
                              const double* eps, int64_t nbf, int64_t nocc, int64_t i0,
                              int64_t ni, double eta, double* R) {
  const int64_t nv = nbf - nocc, ntb = ni * nv;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbf * nocc * ntb) return;
  const int64_t ap = idx % nv;
  int64_t r = idx / nv;
  const int64_t ii = r % ni;
  r /= ni;
  const int64_t p = r % nocc;
  const int64_t n = r / nocc;
  const int64_t i = i0 + ii;
  const int64_t o = (n * nbf + p) * ntb + ii * nv + ap;
  const double x = eps[n] + eps[nocc + ap] - eps[i] - eps[p];
  const double X = xo[n * xsn + i * xsi + p * nv + ap];
  R[o] = (2.0 * D[o] - X) * (x / (x * x + eta * eta));
}

// Right operand for empty p, p' = p - nocc: the exchange integral
// (pi|an) = (na|ip) = D[n][a][ii nv + p'] is the transpose, in (a', p'), of
// the direct block, so each workgroup moves one 32 x 32 tile of it through LDS:
//   Rh[n][p][tb] = (2 (np|ia) - (pi|an)) x / (x^2 + eta^2),
//   x = eps_n + eps_i - eps_a - eps_p.
// Grid: (tiles of (p', a'), ii, n); 256 threads.
__global__ void k_mp2_rhs_vir(const double* D, const double* eps, int64_t nbf, int64_t nocc,
                              int64_t i0, int64_t ni, double eta, double* R) {
  __shared__ double X[32][33];
  const int64_t nv = nbf - nocc, ntb = ni * nv;
  const int64_t nvt = (nv + 31) / 32;
  const int64_t pt = blockIdx.x / nvt, at = blockIdx.x - pt * nvt;
  const int64_t ii = blockIdx.y, n = blockIdx.z;
  const int64_t p0 = pt * 32, a0 = at * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double* Dn = D + n * nbf * ntb + ii * nv;
  for (int r = ty; r < 32; r += 8) {
    const int64_t a = a0 + r, pp = p0 + tx;
    if (a < nv && pp < nv) X[r][tx] = Dn[(nocc + a) * ntb + pp];
  }
  __syncthreads();
  const double en = eps[n], ei = eps[i0 + ii];
  for (int r = ty; r < 32; r += 8) {
    const int64_t pp = p0 + r, a = a0 + tx;
    if (pp < nv && a < nv) {
      const int64_t o = (nocc + pp) * ntb + a;
      const double x = en + ei - eps[nocc + a] - eps[nocc + pp];
      R[n * nbf * ntb + ii * nv + o] = (2.0 * Dn[o] - X[tx][r]) * (x / (x * x + eta * eta));
    }
  }
}

// Open shell: one spin's block of the concatenated transition tensor,
// bt[P * ld + t] = B_mo[P][i][a] sqrt_delta[t] scale, t = (i, a) of that spin.
__global__ void k_gather_bia_ld(const double* bmo, const double* sqrt_delta, double scale,
                                int64_t naux, int64_t nbf, int64_t nocc, int64_t ld, double* bt) {
  const int64_t nv = nbf - nocc;
  const int64_t ntr = nocc * nv;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= naux * ntr) return;
  const int64_t P = idx / ntr;
  const int64_t t = idx - P * ntr;
  const int64_t i = t / nv;
  const int64_t a = nocc + (t - i * nv);
  bt[P * ld + t] = bmo[(P * nbf + i) * nbf + a] * sqrt_delta[t] * scale;
}

}  // namespace qsgw
