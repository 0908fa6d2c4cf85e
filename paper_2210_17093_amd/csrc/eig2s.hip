// Two-stage dense symmetric eigensolver for the Casida problem M Z = Z Omega^2
// (Eq. (12) in its Hermitian form).  The one-stage reduction to tridiagonal
// form reads the whole trailing matrix once per column (matrix-vector
// products, bound by HBM bandwidth); here the reduction goes through a band
// of half-width b so that almost all of its work is matrix-matrix products:
//
//   1. dense -> band: for each panel of b columns, a Householder QR of the
//      part below the band (V, T with H = I - V T V^T) and the two-sided
//      update S <- H^T S H of the trailing matrix as matrix products
//      (X = S V T, W = X - 1/2 V (T^T V^T X), S -= V W^T + W V^T);
//   2. band -> tridiagonal: bulge chasing.  Sweep i annihilates column i
//      below the first sub-diagonal with a reflector on rows i+1..i+b, and
//      each step k >= 1 re-applies the previous reflector to the block of
//      rows [i+1+kb, i+(k+1)b] it fills, annihilates that block's first
//      column and applies the new reflector to the diagonal block.  Step k
//      of sweep i runs at time 3i + k: the steps sharing a time touch
//      disjoint columns of the band, so each time is one launch with one
//      workgroup per step, and the result equals the sweep-by-sweep order;
//   3. tridiagonal eigenproblem: rocSOLVER divide and conquer (dstedc),
//      eigenvectors E of the tridiagonal matrix;
//   4. back-transformations Z = Q1 Q2 E: the bulge-chasing reflectors in
//      blocks of g consecutive sweeps at one step k (block (J, k) needs
//      (J+1, k) and (J, k-1), so the blocks of one anti-diagonal are
//      independent and touch disjoint rows), then the panel reflectors with
//      rocSOLVER larfb (matrix products).
//
// All arrays are column-major; a symmetric row-major matrix is its own
// column-major view.  Everything runs in FP64.
#include "internal.hpp"

namespace {

constexpr int kBand = 64;  // band half-width b (and the sweep group size g)

// ------------------------------------------------------------- helpers ----
__device__ __forceinline__ double quad_sum(double x) {
  // sum over the 4 consecutive lanes that share a row or column
  x += __shfl_xor(x, 1);
  x += __shfl_xor(x, 2);
  return x;
}

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Copies the panel's Householder vectors (below the diagonal of the geqrf
// output, unit diagonal implied) into V [m][kk] column-major (ld m) with an
// explicit unit diagonal and zeros above it, and into the concatenated
// operands U1 = [V | W] (columns 0..kk-1) and U2 = [W | V] (columns kk..2kk-1).
__global__ void k_panel_v(const double* __restrict__ P, int64_t lda, int64_t m, int64_t kk,
                          double* __restrict__ V, double* __restrict__ U1,
                          double* __restrict__ U2) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * kk) return;
  const int64_t col = idx / m, r = idx - col * m;
  const double v = r > col ? P[col * lda + r] : (r == col ? 1.0 : 0.0);
  V[idx] = v;
  U1[idx] = v;
  U2[kk * m + idx] = v;
}

// Lower band of the reduced matrix: AB[c][d] = A[c + d][c] for d <= b, 0 for
// b < d < ldab (room for the bulges of stage 2).
__global__ void k_band_extract(const double* __restrict__ A, int64_t n, int b, int64_t ldab,
                               double* __restrict__ AB) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ldab) return;
  const int64_t c = idx / ldab, d = idx - c * ldab;
  AB[idx] = (d <= b && c + d < n) ? A[c * n + c + d] : 0.0;
}

__global__ void k_tridiag(const double* __restrict__ AB, int64_t n, int64_t ldab,
                          double* __restrict__ dd, double* __restrict__ ee) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  dd[c] = AB[c * ldab];
  if (c + 1 < n) ee[c] = AB[c * ldab + 1];
}

// Householder reflector of x[0..L) held in x (shared): on return v[0..kBand)
// (v[0] = 1, zero past L), *tau and *beta with (I - tau v v^T) x = beta e_1.
// Called by the whole workgroup; wave 0 reduces.
__device__ void householder(const double* x, int L, double* v, double* sc) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const double xv = (tid >= 1 && tid < L) ? x[tid] : 0.0;
    const double s = wave_sum(xv * xv);
    if (tid == 0) {
      const double alpha = x[0];
      if (s == 0.0) {
        sc[0] = 0.0;     // tau: H = I
        sc[1] = alpha;   // beta
        sc[2] = 0.0;     // scale of x[1:]
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + s), alpha);
        sc[0] = (beta - alpha) / beta;
        sc[1] = beta;
        sc[2] = 1.0 / (alpha - beta);
      }
    }
  }
  __syncthreads();
  if (tid < kBand) v[tid] = tid == 0 ? 1.0 : (tid < L ? x[tid] * sc[2] : 0.0);
  __syncthreads();
}

// One bulge-chasing step (i, k) with k = t - 3 i, one workgroup each.
// AB: lower band storage, AB[c * ldab + d] = A[c + d][c], ldab >= 2b.
// V2/tau2: the reflector of step (i, k) at V2[(off[i] + k) * b], tau2[off[i] + k].
__global__ __launch_bounds__(256) void k_bulge(double* __restrict__ AB, int64_t ldab, int64_t n,
                                               int b, double* __restrict__ V2,
                                               double* __restrict__ tau2,
                                               const int64_t* __restrict__ off, int64_t t,
                                               int64_t i_lo) {
  const int64_t i = i_lo + blockIdx.x;
  const int64_t k = t - 3 * i;
  if (i > n - 3 || k < 0) return;
  const int64_t K = (n - 1 - i + b - 1) / b;
  if (k >= K) return;
  __shared__ double O[kBand][kBand + 1];
  __shared__ double D[kBand][kBand + 1];
  __shared__ double v[kBand], vp[kBand], y[kBand], x[kBand];
  __shared__ double sc[4];
  const int tid = threadIdx.x;
  const int q = tid & 3, rr = tid >> 2;  // 4 lanes per row (or column) rr
  const int64_t r0 = i + 1 + k * b;
  const int64_t r1 = min(i + (k + 1) * b, n - 1);
  const int L = (int)(r1 - r0 + 1);

  if (k == 0) {
    if (tid < kBand) x[tid] = tid < L ? AB[i * ldab + 1 + tid] : 0.0;
    __syncthreads();
    householder(x, L, v, sc);
    if (tid < L) AB[i * ldab + 1 + tid] = tid == 0 ? sc[1] : 0.0;
  } else {
    const int64_t p0 = i + 1 + (k - 1) * b;  // the previous window (always b long)
    for (int e = tid; e < kBand * kBand; e += 256) {
      const int c = e / kBand, a = e - c * kBand;  // consecutive threads: consecutive rows
      O[a][c] = (a < L && c < b) ? AB[(p0 + c) * ldab + (b + a - c)] : 0.0;
    }
    if (tid < kBand) vp[tid] = tid < b ? V2[(off[i] + k - 1) * b + tid] : 0.0;
    if (tid == 0) sc[3] = tau2[off[i] + k - 1];
    __syncthreads();
    // O <- O (I - taup vp vp^T)
    {
      double s = 0.0;
      for (int c = q; c < kBand; c += 4) s += O[rr][c] * vp[c];
      s = quad_sum(s);
      if (q == 0) y[rr] = s;
    }
    __syncthreads();
    const double taup = sc[3];
    for (int e = tid; e < kBand * kBand; e += 256) {
      const int a = e / kBand, c = e - a * kBand;
      O[a][c] -= taup * y[a] * vp[c];
    }
    __syncthreads();
    if (tid < kBand) x[tid] = O[tid][0];
    __syncthreads();
    householder(x, L, v, sc);
    const double tau = sc[0];
    // first column -> beta e_1; the other columns <- H O
    {
      double s = 0.0;
      for (int a = q; a < kBand; a += 4) s += v[a] * O[a][rr];
      s = quad_sum(s);
      if (q == 0) y[rr] = s;
    }
    __syncthreads();
    for (int e = tid; e < kBand * kBand; e += 256) {
      const int a = e / kBand, c = e - a * kBand;
      if (c == 0)
        O[a][0] = a == 0 ? sc[1] : 0.0;
      else
        O[a][c] -= tau * v[a] * y[c];
    }
    __syncthreads();
    for (int e = tid; e < kBand * kBand; e += 256) {
      const int c = e / kBand, a = e - c * kBand;
      if (a < L && c < b) AB[(p0 + c) * ldab + (b + a - c)] = O[a][c];
    }
  }
  // diagonal block D <- H D H on rows/columns r0..r1
  // lower triangle from the band (consecutive threads: consecutive rows), then mirrored
  for (int e = tid; e < kBand * kBand; e += 256) {
    const int c = e / kBand, a = e - c * kBand;
    if (a >= c) D[a][c] = (a < L) ? AB[(r0 + c) * ldab + (a - c)] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < kBand * kBand; e += 256) {
    const int c = e / kBand, a = e - c * kBand;
    if (a < c) D[a][c] = D[c][a];
  }
  __syncthreads();
  const double tau = sc[0];
  {
    double s = 0.0;
    for (int c = q; c < kBand; c += 4) s += D[rr][c] * v[c];
    s = quad_sum(s);
    if (q == 0) y[rr] = tau * s;
  }
  __syncthreads();
  if (tid < 64) {
    const double wv = wave_sum(y[tid] * v[tid]);
    if (tid == 0) sc[2] = -0.5 * tau * wv;
  }
  __syncthreads();
  const double al = sc[2];
  for (int e = tid; e < kBand * kBand; e += 256) {
    const int c = e / kBand, a = e - c * kBand;
    if (a < L && c <= a) {
      const double wa = y[a] + al * v[a], wc = y[c] + al * v[c];
      AB[(r0 + c) * ldab + (a - c)] = D[a][c] - v[a] * wc - wa * v[c];
    }
  }
  if (tid < b) V2[(off[i] + k) * b + tid] = v[tid];
  if (tid == 0) tau2[off[i] + k] = tau;
}

// Compact WY factor of block (J, k) of the bulge-chasing reflectors: with V
// column o the reflector of sweep c = J g + o at step k (rows o..o+b-1 of the
// block), H_{Jg} H_{Jg+1} ... H_{Jg+g-1} = I - V T V^T, T upper triangular
// (T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] V[:, 0:j]^T v_j).  Missing
// reflectors (past the last sweep, or sweeps that end before step k) have
// tau = 0.  Tb: [blocks][64][64], block (J, k) at boff[J] + k.
__global__ __launch_bounds__(256) void k_q2_tfactor(const double* __restrict__ V2,
                                                    const double* __restrict__ tau2,
                                                    const int64_t* __restrict__ off,
                                                    const int64_t* __restrict__ boff, int64_t n,
                                                    int b, double* __restrict__ Tb) {
  const int64_t J = blockIdx.x, k = blockIdx.y;
  const int g = b;
  const int64_t c_lo = J * g;
  const int64_t c_hi = min(c_lo + g, n - 2) - 1;
  if (c_hi < c_lo || k >= (n - 1 - c_lo + b - 1) / b) return;
  __shared__ double Vb[kBand][kBand + 1];
  __shared__ double G[kBand][kBand + 1];
  __shared__ double T[kBand][kBand + 1];
  __shared__ double ts[kBand];
  const int tid = threadIdx.x;
  for (int e = tid; e < kBand * kBand; e += 256) {
    const int o = e / kBand, a = e - o * kBand;
    const int64_t c = c_lo + o;
    const bool ok = c <= c_hi && k < (n - 1 - c + b - 1) / b && a < b;
    Vb[o][a] = ok ? V2[(off[c] + k) * b + a] : 0.0;
    T[o][a] = 0.0;
  }
  if (tid < kBand) {
    const int64_t c = c_lo + tid;
    ts[tid] = (c <= c_hi && k < (n - 1 - c + b - 1) / b) ? tau2[off[c] + k] : 0.0;
  }
  __syncthreads();
  // G[i][j] = v_i . v_j (i < j): v_i starts at row i, v_j at row j
  for (int e = tid; e < kBand * kBand; e += 256) {
    const int i = e / kBand, j = e - i * kBand;
    double sum = 0.0;
    if (i < j)
      for (int a = j - i; a < kBand; ++a) sum += Vb[i][a] * Vb[j][a - (j - i)];
    G[i][j] = sum;
  }
  __syncthreads();
  for (int j = 0; j < kBand; ++j) {
    if (tid < j) {
      double sum = 0.0;
      for (int l = tid; l < j; ++l) sum += T[tid][l] * G[l][j];
      T[tid][j] = -ts[j] * sum;
    } else if (tid == j) {
      T[j][j] = ts[j];
    }
    __syncthreads();
  }
  double* out = Tb + (boff[J] + k) * (kBand * kBand);
  for (int e = tid; e < kBand * kBand; e += 256) out[e] = T[e / kBand][e % kBand];
}

// X <- B X for the blocks (J, k) of one anti-diagonal t = (nJ - 1 - J) + k on
// a slab of kSlabW columns of X ([n][ncols] column-major, ld n):
//   trans 0: B = I - V T V^T   (the block's reflectors from its highest sweep
//            down; anti-diagonals in ascending order give X <- Q2 X);
//   trans 1: B = I - V T^T V^T (lowest sweep first; anti-diagonals in
//            descending order give X <- Q2^T X).
// The block touches rows [J g + 1 + k b, J g + g - 1 + (k + 1) b] of X.
constexpr int kSlabW = 32;
constexpr int kRows = 2 * kBand;  // b + g - 1 rows, padded
__global__ __launch_bounds__(256) void k_q2_apply(double* __restrict__ X, int64_t n, int64_t ncols,
                                                  int b, const double* __restrict__ V2,
                                                  const int64_t* __restrict__ off,
                                                  const double* __restrict__ Tb,
                                                  const int64_t* __restrict__ boff, int64_t t,
                                                  int64_t nJ, int64_t J_lo, int64_t nslab,
                                                  int trans) {
  const int64_t jj = blockIdx.x / nslab, slab = blockIdx.x - jj * nslab;
  const int64_t J = J_lo + jj;
  const int64_t k = t - (nJ - 1 - J);
  if (J >= nJ || k < 0) return;
  const int g = b;
  const int64_t c_lo = J * g;
  const int64_t c_hi = min(c_lo + g, n - 2) - 1;
  if (c_hi < c_lo || k >= (n - 1 - c_lo + b - 1) / b) return;
  __shared__ double Eb[kRows][kSlabW + 1];
  __shared__ double Vb[kBand][kBand + 1];
  __shared__ double Ts[kBand][kBand + 1];
  __shared__ double W[kBand][kSlabW + 1];
  __shared__ double W2[kBand][kSlabW + 1];
  const int tid = threadIdx.x;
  const int64_t R0 = c_lo + 1 + k * b;
  const int64_t R1 = min(c_hi + (k + 1) * b, n - 1);
  const int NR = (int)(R1 - R0 + 1);
  const int64_t col0 = slab * kSlabW;
  const int ncol = (int)min((int64_t)kSlabW, ncols - col0);
  for (int e = tid; e < kSlabW * kRows; e += 256) {
    const int cl = e / kRows, r = e - cl * kRows;  // consecutive threads: consecutive rows
    Eb[r][cl] = (cl < ncol && r < NR) ? X[(col0 + cl) * n + R0 + r] : 0.0;
  }
  const double* Tg = Tb + (boff[J] + k) * (kBand * kBand);
  for (int e = tid; e < kBand * kBand; e += 256) {
    const int o = e / kBand, a = e - o * kBand;
    const int64_t c = c_lo + o;
    const bool ok = c <= c_hi && k < (n - 1 - c + b - 1) / b && a < b;
    Vb[o][a] = ok ? V2[(off[c] + k) * b + a] : 0.0;
    Ts[o][a] = Tg[e];
  }
  __syncthreads();
  const int cl = tid & (kSlabW - 1), grp = tid / kSlabW;  // 8 groups of 8 reflectors
  // W = V^T X_block: W[o][c] = sum_a Vb[o][a] Eb[o + a][c]
  {
    double acc[8], e8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc[u] = 0.0;
      e8[u] = Eb[grp * 8 + u][cl];
    }
    for (int a = 0; a < kBand; ++a) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += Vb[grp * 8 + u][a] * e8[u];
#pragma unroll
      for (int u = 0; u < 7; ++u) e8[u] = e8[u + 1];
      e8[7] = Eb[grp * 8 + 8 + a][cl];  // row grp*8 + 7 + (a + 1) <= 127
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) W[grp * 8 + u][cl] = acc[u];
  }
  __syncthreads();
  // W2 = T W or T^T W
  {
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int j = 0; j < kBand; ++j) {
      const double wj = W[j][cl];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = grp * 8 + u;
        acc[u] += (trans ? Ts[j][i] : Ts[i][j]) * wj;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) W2[grp * 8 + u][cl] = acc[u];
  }
  __syncthreads();
  // X_block -= V W2: row r gets sum over o with 0 <= r - o < b of Vb[o][r - o] W2[o][c]
  {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int o = 0; o < kBand; ++o) {
      const double w2 = W2[o][cl];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int a = grp * 16 + u - o;
        const double v = (a >= 0 && a < kBand) ? Vb[o][a & (kBand - 1)] : 0.0;
        acc[u] += v * w2;
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) Eb[grp * 16 + u][cl] -= acc[u];
  }
  __syncthreads();
  for (int e = tid; e < kSlabW * kRows; e += 256) {
    const int c2 = e / kRows, r = e - c2 * kRows;
    if (c2 < ncol && r < NR) X[(col0 + c2) * n + R0 + r] = Eb[r][c2];
  }
}

#define RB_TRY(ctx, expr, what)                                                           \
  do {                                                                                    \
    rocblas_status s_ = (expr);                                                           \
    if (s_ != rocblas_status_success)                                                     \
      return fail(ctx, QSGW_ERR_SOLVER, "%s: %s returned rocblas status %d", what, #expr, \
                  (int)s_);                                                               \
  } while (0)

// State of one two-stage reduction kept for the back-transformations (the
// reflectors themselves live in the context workspace).
struct TwoStage {
  std::vector<int64_t> pj, pm, poff;  // panels: first column, rows below the band, offset in V1
  int64_t np = 0, nJ = 0, K0 = 0;
  double *V1 = nullptr, *T1 = nullptr, *V2 = nullptr, *tau2 = nullptr, *Tb = nullptr;
  int64_t* off = nullptr;  // first step of each sweep, then the first block of each group
};

// Stages 1-3: A [n][n] symmetric in; on return A holds the eigenvectors E of the
// tridiagonal matrix (column-major) and evals the eigenvalues, ascending.
static int ts_reduce(qsgw_ctx* c, int64_t n, double* A, double* evals, const char* what,
                     TwoStage* ts) {
  const int b = kBand;
  rocblas_handle h = c->blas;
  const int ni = (int)n;

  // ---- stage 1: dense -> band ----
  int64_t vtot = 0;
  for (int64_t j = 0; n - j - b > 1; j += b) {
    ts->pj.push_back(j);
    ts->pm.push_back(n - j - b);
    ts->poff.push_back(vtot);
    vtot += (n - j - b) * b;
  }
  const int64_t np = ts->np = (int64_t)ts->pj.size();
  double *V1, *T1, *tau1, *U1, *U2, *X, *Y, *Z1, *Z2, *AB, *V2, *tau2, *dd, *ee;
  int64_t* off;
  int* flags;
  CHECK(ws_get(c, W_EIG_V1, (size_t)vtot, &V1));
  CHECK(ws_get(c, W_EIG_T1, (size_t)(np * b * b), &T1));
  CHECK(ws_get(c, W_EIG_TAU1, (size_t)(np * b), &tau1));
  CHECK(ws_get(c, W_EIG_U, (size_t)(4 * n * b), &U1));
  U2 = U1 + 2 * n * b;
  CHECK(ws_get(c, W_EIG_XY, (size_t)(2 * n * b + 2 * b * b), &X));
  Y = X + n * b;
  Z1 = Y + n * b;
  Z2 = Z1 + b * b;
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  const double one = 1.0, zero = 0.0, mone = -1.0, mhalf = -0.5;
  for (int64_t p = 0; p < np; ++p) {
    const int64_t j = ts->pj[p], m = ts->pm[p], kk = m < b ? m : b;
    const int mi = (int)m, ki = (int)kk;
    double* P = A + j * n + (j + b);
    double* S = A + (j + b) * n + (j + b);
    double* V = V1 + ts->poff[p];
    double* T = T1 + p * b * b;
    RB_TRY(c, rocsolver_dgeqrf(h, mi, b, P, ni, tau1 + p * b), what);
    hipLaunchKernelGGL(k_panel_v, dim3(blocks_for(m * kk)), dim3(256), 0, c->stream, P, n, m, kk,
                       V, U1, U2);
    CHECK(launch_check(c, "k_panel_v"));
    RB_TRY(c, rocsolver_dlarft(h, rocblas_forward_direction, rocblas_column_wise, mi, ki, V, mi,
                               tau1 + p * b, T, b), what);
    // Y = V T;  X = S Y;  Z1 = V^T X;  Z2 = T^T Z1;  W = X - 1/2 V Z2 (in X)
    RB_TRY(c, rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, mi, ki, ki, &one, V,
                            mi, T, b, &zero, Y, mi), what);
    RB_TRY(c, rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, mi, ki, mi, &one, S,
                            ni, Y, mi, &zero, X, mi), what);
    RB_TRY(c, rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, ki, ki, mi, &one,
                            V, mi, X, mi, &zero, Z1, b), what);
    RB_TRY(c, rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, ki, ki, ki, &one,
                            T, b, Z1, b, &zero, Z2, b), what);
    RB_TRY(c, rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, mi, ki, ki, &mhalf, V,
                            mi, Z2, b, &one, X, mi), what);
    // S -= [V W] [W V]^T
    HIP_TRY(c, hipMemcpyAsync(U1 + kk * m, X, (size_t)(m * kk) * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(U2, X, (size_t)(m * kk) * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    RB_TRY(c, rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, mi, mi, 2 * ki,
                            &mone, U1, mi, U2, mi, &one, S, ni), what);
  }

  // ---- stage 2: band -> tridiagonal ----
  const int64_t ldab = 2 * b + 1;
  std::vector<int64_t> hoff((size_t)n, 0);
  int64_t nref = 0, tmax = 0;
  for (int64_t i = 0; i <= n - 3; ++i) {
    hoff[(size_t)i] = nref;
    const int64_t K = (n - 1 - i + b - 1) / b;
    nref += K;
    if (3 * i + K > tmax) tmax = 3 * i + K;
  }
  const int64_t nJ = ts->nJ = (n - 2 + b - 1) / b;  // groups of g = b sweeps
  const int64_t K0 = ts->K0 = (n - 1 + b - 1) / b;
  // block (J, k) of the back-transformation: its T factor at boff[J] + k
  int64_t nblk = 0;
  for (int64_t J = 0; J < nJ; ++J) {
    hoff.push_back(nblk);
    nblk += (n - 1 - J * b + b - 1) / b;
  }
  CHECK(ws_get(c, W_EIG_BAND, (size_t)(ldab * n), &AB));
  CHECK(ws_get(c, W_EIG_V2, (size_t)(nref * b), &V2));
  CHECK(ws_get(c, W_EIG_TAU2, (size_t)nref, &tau2));
  CHECK(ws_get(c, W_EIG_OFF, (size_t)(n + nJ), &off));
  CHECK(ws_get(c, W_EIG_DE, (size_t)(2 * n), &dd));
  CHECK(ws_get(c, W_EIG_TB, (size_t)(nblk * b * b), &ts->Tb));
  ee = dd + n;
  // (pointers into slots sized above; no slot is resized after this)
  ts->V1 = static_cast<double*>(c->ws[W_EIG_V1].p);
  ts->T1 = static_cast<double*>(c->ws[W_EIG_T1].p);
  ts->V2 = V2;
  ts->tau2 = tau2;
  ts->off = off;
  HIP_TRY(c, hipMemcpyAsync(off, hoff.data(), (size_t)(n + nJ) * sizeof(int64_t),
                            hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_band_extract, dim3(blocks_for(n * ldab)), dim3(256), 0, c->stream, A, n, b,
                     ldab, AB);
  CHECK(launch_check(c, "k_band_extract"));
  for (int64_t t = 0; t < tmax; ++t) {
    int64_t i_hi = t / 3;
    if (i_hi > n - 3) i_hi = n - 3;
    int64_t i_lo = t - K0 >= 0 ? (t - K0) / 3 + 1 : 0;  // 3 i > t - K0
    if (i_lo > i_hi) continue;
    hipLaunchKernelGGL(k_bulge, dim3((unsigned)(i_hi - i_lo + 1)), dim3(256), 0, c->stream, AB,
                       ldab, n, b, V2, tau2, off, t, i_lo);
  }
  CHECK(launch_check(c, "k_bulge"));
  hipLaunchKernelGGL(k_tridiag, dim3(blocks_for(n)), dim3(256), 0, c->stream, AB, n, ldab, dd, ee);
  CHECK(launch_check(c, "k_tridiag"));
  hipLaunchKernelGGL(k_q2_tfactor, dim3((unsigned)nJ, (unsigned)K0), dim3(256), 0, c->stream, V2,
                     tau2, off, off + n, n, b, ts->Tb);
  CHECK(launch_check(c, "k_q2_tfactor"));

  // ---- stage 3: tridiagonal eigenproblem (eigenvectors E into A) ----
  RB_TRY(c, rocsolver_dstedc(h, rocblas_evect_tridiagonal, ni, dd, ee, A, ni,
                             (rocblas_int*)(flags + 1)), what);
  int info = 0;
  CHECK(read_flag(c, flags + 1, &info));
  if (info != 0) return fail(c, QSGW_ERR_SOLVER, "%s: dstedc info = %d", what, info);
  HIP_TRY(c, hipMemcpyAsync(evals, dd, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
  return QSGW_OK;
}

// X [n][ncols] column-major (ld n) <- Q1 Q2 X (trans false) or Q2^T Q1^T X (trans true).
static int ts_apply(qsgw_ctx* c, const TwoStage& ts, int64_t n, double* X, int64_t ncols, bool trans,
                    const char* what) {
  const int b = kBand;
  const int ni = (int)n, nc = (int)ncols;
  const int64_t nslab = (ncols + kSlabW - 1) / kSlabW;
  auto q2 = [&](int64_t t) {
    // blocks J with 0 <= k = t - (nJ - 1 - J) < K0
    int64_t J_lo = ts.nJ - 1 - t;
    if (J_lo < 0) J_lo = 0;
    int64_t J_hi = ts.nJ - 1 - t + (ts.K0 - 1);
    if (J_hi > ts.nJ - 1) J_hi = ts.nJ - 1;
    if (J_hi < J_lo) return;
    hipLaunchKernelGGL(k_q2_apply, dim3((unsigned)((J_hi - J_lo + 1) * nslab)), dim3(256), 0,
                       c->stream, X, n, ncols, b, ts.V2, ts.off, ts.Tb, ts.off + n, t, ts.nJ, J_lo,
                       nslab, trans ? 1 : 0);
  };
  auto q1 = [&](int64_t p) -> int {
    const int64_t j = ts.pj[(size_t)p], m = ts.pm[(size_t)p], kk = m < b ? m : b;
    RB_TRY(c, rocsolver_dlarfb(c->blas, rocblas_side_left,
                               trans ? rocblas_operation_transpose : rocblas_operation_none,
                               rocblas_forward_direction, rocblas_column_wise, (int)m, nc, (int)kk,
                               ts.V1 + ts.poff[(size_t)p], (int)m, ts.T1 + p * b * b, b,
                               X + (j + b), ni), what);
    return QSGW_OK;
  };
  if (!trans) {
    for (int64_t t = 0; t < ts.nJ + ts.K0; ++t) q2(t);
    CHECK(launch_check(c, "k_q2_apply"));
    for (int64_t p = ts.np - 1; p >= 0; --p) CHECK(q1(p));
  } else {
    for (int64_t p = 0; p < ts.np; ++p) CHECK(q1(p));
    for (int64_t t = ts.nJ + ts.K0 - 1; t >= 0; --t) q2(t);
    CHECK(launch_check(c, "k_q2_apply"));
  }
  return QSGW_OK;
}

}  // namespace

// Two-stage eigensolve: A [n][n] symmetric (column-major view) in, its
// eigenvectors column-major out (column s for evals[s], ascending).
int eig_two_stage(qsgw_ctx* c, int64_t n, double* A, double* evals, const char* what) {
  if (n > 46340) return fail(c, QSGW_ERR_UNSUPPORTED, "%s: n too large for the two-stage solver", what);
  if (n < 4 * kBand) return syevd(c, n, A, evals, what);
  TwoStage ts;
  CHECK(ts_reduce(c, n, A, evals, what, &ts));
  return ts_apply(c, ts, n, A, n, false, what);
}

// Eigenvalues of A and the projection R = Z^T Bt^T of a row-major [naux][n]
// matrix Bt on the eigenvectors Z, written as row-major [naux][n] (R[P][s] =
// sum_t Bt[P][t] Z[t][s]), without forming Z: the back-transformations act on
// the naux columns of Bt^T instead of the n columns of E,
//   R^T = E^T (Q2^T Q1^T Bt^T).
// A is destroyed (it holds E on return); X: [naux][n] work array.
int eig_two_stage_project(qsgw_ctx* c, int64_t n, double* A, double* evals, int64_t naux,
                          const double* Bt, double* X, double* R, const char* what) {
  if (n > 46340) return fail(c, QSGW_ERR_UNSUPPORTED, "%s: n too large for the two-stage solver", what);
  if (naux > 0x7fffffffLL) return fail(c, QSGW_ERR_UNSUPPORTED, "%s: naux too large", what);
  const double one = 1.0, zero = 0.0;
  const double* Xp = Bt;
  if (n < 4 * kBand) {
    CHECK(syevd(c, n, A, evals, what));  // A = Z
  } else {
    TwoStage ts;
    CHECK(ts_reduce(c, n, A, evals, what, &ts));
    HIP_TRY(c, hipMemcpyAsync(X, Bt, (size_t)(naux * n) * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    CHECK(ts_apply(c, ts, n, X, naux, true, what));
    Xp = X;
  }
  RB_TRY(c, rocblas_dgemm(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)n,
                          (int)naux, (int)n, &one, A, (int)n, Xp, (int)n, &zero, R, (int)n), what);
  return QSGW_OK;
}
