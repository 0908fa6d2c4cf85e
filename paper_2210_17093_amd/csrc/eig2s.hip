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
//      of sweep i runs at time 2i + k: the steps sharing a time touch
//      disjoint rows of the band, so each time is one launch with one
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

// Householder QR of one panel (m x b, column-major, ld lda), one launch per
// column j with a partition of the rows over the workgroups (256 RPT rows
// each: RPT = 1 spreads a panel of up to 16,384 rows over at least 64
// compute units, RPT = 2 halves the partial sums of taller panels).  Column j's reflector needs dots[c] = sum_{r > j} P[r][j] P[r][c]
// (c >= j) of the current panel: the launch for column j - 1 leaves one
// partial sum per workgroup (part_in[g][c]) and every workgroup of the launch
// for column j adds them up in a fixed order.  Then, with the LAPACK dlarfg
// convention (v_j = 1, beta = -sign(alpha) |x|, tau = (beta - alpha) / beta),
//   w_c = P[j][c] + dots[c] / (alpha - beta)      (w = v^T P[:, c]),
//   P[r][j] <- v_r = P[r][j] / (alpha - beta),  P[r][c] -= tau v_r w_c  (r > j, c > j),
// and row j of R goes to Rbuf (P's row j is left as it was: every workgroup
// reads it).  Each workgroup then leaves its partial dots for column j + 1.
// j = -1 only computes the partial dots of column 0.
template <int RPT>
__global__ __launch_bounds__(256) void k_panel_col(double* __restrict__ P, int64_t lda, int64_t m,
                                                   int b, int j, const double* __restrict__ part_in,
                                                   double* __restrict__ part_out, int G,
                                                   double* __restrict__ Rbuf,
                                                   double* __restrict__ tau) {
  __shared__ double wv[kBand];
  __shared__ double sc[3];
  __shared__ double red[4][kBand];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x;
  const int64_t rbase = (int64_t)g * (256 * RPT);
  if (j >= 0) {
    // column j's dots from the previous launch's partial sums
    if (tid < kBand) {
      double s2 = 0.0;
      if (tid >= j && tid < b)
        for (int h = 0; h < G; ++h) s2 += part_in[(int64_t)h * kBand + tid];
      wv[tid] = s2;
    }
    __syncthreads();
    if (tid == 0) {
      const double alpha = P[(int64_t)j * lda + j];
      const double sig = wv[j];
      if (sig == 0.0) {
        sc[0] = 0.0;
        sc[1] = alpha;
        sc[2] = 0.0;
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + sig), alpha);
        sc[0] = (beta - alpha) / beta;
        sc[1] = beta;
        sc[2] = 1.0 / (alpha - beta);
      }
    }
    __syncthreads();
    const double t = sc[0], scale = sc[2];
    double wc = 0.0;
    if (tid > j && tid < b) wc = P[(int64_t)tid * lda + j] + scale * wv[tid];
    __syncthreads();
    if (tid < kBand) wv[tid] = wc;
    __syncthreads();
    if (g == 0 && tid < kBand) {  // row j of R, and tau
      if (tid == j) Rbuf[(int64_t)j * kBand + j] = sc[1];
      if (tid > j && tid < b) Rbuf[(int64_t)j * kBand + tid] = P[(int64_t)tid * lda + j] - t * wv[tid];
      if (tid == 0) tau[j] = t;
    }
    // rows r > j of this workgroup: v_r into column j, the other columns updated
    double v[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int64_t r = rbase + tid + 256 * u;
      v[u] = 0.0;
      if (r > j && r < m) {
        v[u] = P[(int64_t)j * lda + r] * scale;
        P[(int64_t)j * lda + r] = v[u];
      }
    }
    if (t != 0.0) {
      // columns in chunks of 8: all loads of a chunk first, then the stores
      for (int c0 = j + 1; c0 < b; c0 += 8) {
        double x[8][RPT];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc)
#pragma unroll
          for (int u = 0; u < RPT; ++u) {
            const int64_t r = rbase + tid + 256 * u;
            x[cc][u] = (c0 + cc < b && r > j && r < m) ? P[(int64_t)(c0 + cc) * lda + r] : 0.0;
          }
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          if (c0 + cc >= b) break;
          const double tw = t * wv[c0 + cc];
#pragma unroll
          for (int u = 0; u < RPT; ++u) {
            const int64_t r = rbase + tid + 256 * u;
            if (r > j && r < m) P[(int64_t)(c0 + cc) * lda + r] = x[cc][u] - tw * v[u];
          }
        }
      }
    }
  }
  // partial dots of column j + 1 over this workgroup's rows r > j + 1
  const int jn = j + 1;
  if (jn >= b || jn >= m - 1) return;  // (uniform) no further column to factor here
  double pj[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int64_t r = rbase + tid + 256 * u;
    pj[u] = (r > jn && r < m) ? P[(int64_t)jn * lda + r] : 0.0;
  }
  for (int c0 = jn; c0 < b; c0 += 8) {
    double x[8][RPT];
#pragma unroll
    for (int cc = 0; cc < 8; ++cc)
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int64_t r = rbase + tid + 256 * u;
        x[cc][u] = (c0 + cc < b && r > jn && r < m) ? P[(int64_t)(c0 + cc) * lda + r] : 0.0;
      }
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      double s2 = 0.0;
#pragma unroll
      for (int u = 0; u < RPT; ++u) s2 += pj[u] * x[cc][u];
      s2 = wave_sum(s2);
      if (lane == 0 && c0 + cc < b) red[wave][c0 + cc] = s2;
    }
  }
  __syncthreads();
  if (tid < kBand)
    part_out[(int64_t)g * kBand + tid] =
        (tid >= jn && tid < b) ? red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid] : 0.0;
}

// The same Householder QR of one panel (b = 64 columns) in one cooperative
// launch: workgroup g keeps rows [256 g, 256 g + 256) of the panel in LDS for
// the whole factorisation, and the launches of the per-column kernel become
// grid barriers.  Column j: every workgroup writes its partial dots of column
// j (part[j % 2][g][c], c >= j) and workgroup 0 the panel's row j as updated
// so far (rowj[j % 2][c]); after the barrier every workgroup adds the partial
// dots in the same fixed order, forms the reflector as k_panel_col does and
// applies it to its rows.  Two parities of the exchange buffers let a
// workgroup publish column j + 1 while another still reads column j.  The
// panel goes back to global memory at the end (rows < b as they stand; R
// comes from Rbuf through k_panel_r).
// The barrier: each workgroup stores gen = gen0 + j + 1 into its own flag
// (a release store at agent scope, after a workgroup barrier that has every
// thread's exchange writes done), then threads 0..G-1 each wait for one
// workgroup's flag to reach gen (relaxed agent-scope loads) and the workgroup
// takes an agent-scope acquire fence; no counter is contended.  The
// cooperative launch guarantees that all G workgroups are resident, so every
// flag is eventually written; a wait is still bounded (kPanelSpinMax polls),
// and a workgroup that runs out stops waiting and raises *err, which the host
// turns into an error.  Flags only grow within a solve (gen0 = 64 p for panel
// p) and are cleared before each solve.
constexpr int kPanelSpinMax = 1 << 22;
__global__ __launch_bounds__(256) void k_panel_coop(double* __restrict__ P, int64_t lda, int64_t m,
                                                    double* __restrict__ part,
                                                    double* __restrict__ rowj, int G,
                                                    double* __restrict__ Rbuf,
                                                    double* __restrict__ tau,
                                                    unsigned long long* __restrict__ flags,
                                                    unsigned long long gen0,
                                                    int* __restrict__ err) {
  __shared__ double Ps[kBand][257];  // [column][row of this workgroup], odd pitch
  __shared__ double wv[kBand];
  __shared__ double sc[3];
  __shared__ double red[4][kBand];
  __shared__ int stalled;
  if (threadIdx.x == 0) stalled = 0;
  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t r = (int64_t)g * 256 + tid;
  const bool live = r < m;
#pragma unroll 8
  for (int c = 0; c < kBand; ++c) Ps[c][tid] = live ? P[(int64_t)c * lda + r] : 0.0;
  __syncthreads();
  const int jmax = m - 1 < kBand ? (int)(m - 1) : kBand;  // columns with rows below the diagonal
  for (int j = 0; j < jmax; ++j) {
    const int par = j & 1;
    // partial dots of column j over this workgroup's rows r > j: thread
    // (c = tid % 64, q = tid / 64) sums rows 64 q .. 64 q + 63 of column c in
    // order (rows past m hold zeros; only workgroup 0 has rows r <= j)
    {
      const int cc = tid & 63, qd = tid >> 6;
      double s2 = 0.0;
      if (cc >= j) {
#pragma unroll 8
        for (int u = 0; u < 64; ++u) {
          const int rl = 64 * qd + u;
          const double a = (g > 0 || rl > j) ? Ps[j][rl] : 0.0;
          s2 += a * Ps[cc][rl];
        }
      }
      red[qd][cc] = s2;
    }
    __syncthreads();
    if (tid < kBand) {
      part[((int64_t)par * G + g) * kBand + tid] =
          tid >= j ? red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid] : 0.0;
      if (g == 0) rowj[par * kBand + tid] = Ps[tid][j];  // P[j][tid]: row j < 256 is here
    }
    {
      // grid barrier (see above)
      const unsigned long long gen = gen0 + (unsigned long long)(j + 1);
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(flags + g, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (tid < G && !stalled) {
        int spins = 0;
        while (__hip_atomic_load(flags + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
          if (++spins > kPanelSpinMax) {
            stalled = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    {
      // the same fixed order in every workgroup: four strided partial sums per column
      const int cc = tid & 63, qd = tid >> 6;
      double s2 = 0.0;
      if (cc >= j)
        for (int h = qd; h < G; h += 4) s2 += part[((int64_t)par * G + h) * kBand + cc];
      red[qd][cc] = s2;
    }
    __syncthreads();
    if (tid < kBand) wv[tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    __syncthreads();
    if (tid == 0) {
      const double alpha = rowj[par * kBand + j];
      const double sig = wv[j];
      if (sig == 0.0) {
        sc[0] = 0.0;
        sc[1] = alpha;
        sc[2] = 0.0;
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + sig), alpha);
        sc[0] = (beta - alpha) / beta;
        sc[1] = beta;
        sc[2] = 1.0 / (alpha - beta);
      }
    }
    __syncthreads();
    const double t = sc[0], scale = sc[2];
    double wc = 0.0;
    if (tid > j && tid < kBand) wc = rowj[par * kBand + tid] + scale * wv[tid];
    __syncthreads();
    if (tid < kBand) wv[tid] = wc;
    __syncthreads();
    if (g == 0 && tid < kBand) {  // row j of R, and tau
      if (tid == j) Rbuf[(int64_t)j * kBand + j] = sc[1];
      if (tid > j) Rbuf[(int64_t)j * kBand + tid] = rowj[par * kBand + tid] - t * wv[tid];
      if (tid == 0) tau[j] = t;
    }
    if (live && r > j) {
      const double v = Ps[j][tid] * scale;
      Ps[j][tid] = v;
      if (t != 0.0)
        for (int c = j + 1; c < kBand; ++c) Ps[c][tid] -= t * wv[c] * v;
    }
    __syncthreads();
  }
  if (live) {
#pragma unroll 8
    for (int c = 0; c < kBand; ++c) P[(int64_t)c * lda + r] = Ps[c][tid];
  }
  if (tid == 0 && stalled) atomicOr(err, 1);
}

// R (rows q < b of the panel, columns c >= q) from Rbuf into the panel's upper triangle.
__global__ void k_panel_r(double* __restrict__ P, int64_t lda, int b, const double* __restrict__ Rbuf) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= b * b) return;
  const int q = idx / b, c = idx - q * b;
  if (c >= q) P[(int64_t)c * lda + q] = Rbuf[(int64_t)q * kBand + c];
}

// T factor of a panel's k reflectors from their Gram matrix G[i][j] = v_i . v_j
// (row-major, ld k) and tau, one workgroup: T[j][j] = tau_j,
// T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j] (the forward, column-wise
// convention: H_0 H_1 ... H_{k-1} = I - V T V^T); T column-major, ld ldt.
__global__ __launch_bounds__(256) void k_panel_t(const double* __restrict__ G, int k,
                                                 const double* __restrict__ tau,
                                                 double* __restrict__ T, int ldt) {
  __shared__ double Ts[kBand][kBand + 1];
  __shared__ double Gs[kBand][kBand + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kBand * kBand; e += 256) {
    const int i = e / kBand, l = e % kBand;
    Ts[i][l] = 0.0;
    Gs[i][l] = (i < k && l < k) ? G[i * k + l] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid < j) {
      double sum = 0.0;
      for (int l = tid; l < j; ++l) sum += Ts[tid][l] * Gs[l][j];
      Ts[tid][j] = -tau[j] * sum;
    } else if (tid == j) {
      Ts[j][j] = tau[j];
    }
    __syncthreads();
  }
  for (int e = tid; e < ldt * ldt; e += 256) {
    const int col = e / ldt, row = e - col * ldt;
    T[e] = (row < kBand && col < kBand) ? Ts[row][col] : 0.0;
  }
}

// W = X - 1/2 V Z2 for the panel update, written straight into the second
// half of U1 = [V W] and the first half of U2 = [W V] (both column-major,
// ld m): the element (c, r) of the product W^T handed by the GEMM engine.
struct EpiPanelW {
  const double* X;
  double* U1w;
  double* U2w;
  int64_t m, ldu;
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t c, int64_t r, double v,
                                             bool) const {
    const double w = X[c * m + r] - 0.5 * v;
    U1w[c * ldu + r] = w;
    U2w[c * ldu + r] = w;
  }
};

// A product C[i][c] = sum_r A(i, r) B(c, r) with a long k = r and a small
// output, split over k (partials summed in a fixed order) when that fills
// the chip better; C row-major, ld N.  The k tile is 32 deep: these products
// stream an operand from HBM once, and the deeper tile keeps twice the bytes
// in flight per workgroup.
template <class OA, class OB>
static int gemm_long_k(qsgw_ctx* c, const char* what, OA A, OB B, double* C, int64_t M, int64_t N,
                       int64_t K) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  const SplitPlan sp = round_chunks(split_plan(K, splits_for(tiles, K, 2048)), K, 32);
  if (sp.nz > 1) {
    double* part = nullptr;
    CHECK(ws_get(c, W_EIG_XP, (size_t)(sp.nz * M * N), &part));
    EpiStore E{part, N, 0, M * N, 1.0};
    CHECK((gemm_shape<double, false, 32>(c, SH_64x64, what, A, B, E, M, N, K, 1, sp)));
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks_for(M * N)), dim3(256), 0, c->stream, part, sp.nz,
                       M * N, sp.nz, C);
    return launch_check(c, "k_sum_slices");
  }
  EpiStore E{C, N, 0, 0, 1.0};
  return gemm_shape<double, false, 32>(c, SH_64x64, what, A, B, E, M, N, K, 1);
}

// X[m][n] -= v (a plain product subtracted from its output).
struct EpiSub {
  double* X;
  int64_t ld;
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t m, int64_t n, double v,
                                             bool) const {
    X[m * ld + n] -= v;
  }
};

// X -= C for a symmetric product C computed on the upper tiles only (m <= n,
// a TRI launch): each staged pass of the tile goes out twice, its rows
// (consecutive threads on consecutive columns) for m <= n and its mirror
// X[n][m] (consecutive threads on consecutive rows) for m < n, both coalesced.
// The two halves are disjoint, so X stays exactly symmetric.
struct EpiSubSym {
  static constexpr bool kPassHook = true;
  static constexpr bool kTriPass = true;
  double* X;
  int64_t ld;
  int64_t M;  // order of the product
  template <int ROWS, int BN>
  __device__ __forceinline__ void pass(int64_t r0, int64_t n0, const double* Cs, int ldc,
                                       int tid) const {
    for (int idx = tid; idx < ROWS * BN; idx += 256) {
      const int row = idx / BN, col = idx - (idx / BN) * BN;
      const int64_t m = r0 + row, n = n0 + col;
      if (n < M && m <= n) X[m * ld + n] -= Cs[row * ldc + col];
    }
    for (int idx = tid; idx < ROWS * BN; idx += 256) {
      const int col = idx / ROWS, row = idx - (idx / ROWS) * ROWS;
      const int64_t m = r0 + row, n = n0 + col;
      if (n < M && m < n) X[n * ld + m] -= Cs[row * ldc + col];
    }
  }
};

// Copies the panel's Householder vectors (below the diagonal of the panel QR
// output, unit diagonal implied) into V [m][kk] column-major (ld m) with an
// explicit unit diagonal and zeros above it, and into its two columns blocks of
// the pending-update operands: U1v (the V half of [V W]) and U2v (the V half of
// [W V]), both column-major with ld ldu.
__global__ void k_panel_v(const double* __restrict__ P, int64_t lda, int64_t m, int64_t kk,
                          double* __restrict__ V, double* __restrict__ U1v,
                          double* __restrict__ U2v, int64_t ldu) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * kk) return;
  const int64_t col = idx / m, r = idx - col * m;
  const double v = r > col ? P[col * lda + r] : (r == col ? 1.0 : 0.0);
  V[idx] = v;
  U1v[col * ldu + r] = v;
  U2v[col * ldu + r] = v;
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

// Shared memory of one bulge-chasing step.
struct BulgeSmem {
  double O[kBand][kBand + 1];
  double D[kBand][kBand + 1];
  double v[kBand], vp[kBand], y[kBand], z[kBand], x[kBand], yo[kBand];
  double sc[5];
};

// First step of sweep i in the bulge-chasing reflector arrays: the number of
// steps of the sweeps before it, sum over i' < i of ceil((n - 1 - i') / b),
// in closed form from S(x) = sum_{j = 1..x} ceil(j / b) = b q (q + 1) / 2 + r (q + 1)
// (x = q b + r), so a step needs no table lookup before its reflector loads.
__host__ __device__ __forceinline__ int64_t sweep_first_step(int64_t n, int64_t b, int64_t i) {
  auto S = [b](int64_t x) {
    const int64_t q = x / b, r = x - q * b;
    return b * q * (q + 1) / 2 + r * (q + 1);
  };
  return S(n - 1) - S(n - 1 - i);
}

// One bulge-chasing step (i, k), the whole workgroup (256 threads).
// AB: lower band storage, AB[c * ldab + d] = A[c + d][c], ldab >= 2b.
// V2/tau2: the reflector of step (i, k) at V2[(f + k) * b], tau2[f + k] with f
// the sweep's first step (sweep_first_step).
// Both blocks (the bulge O in the band columns of the previous window, the
// diagonal block D in the columns of this one) are loaded at once: they are
// disjoint.  D is kept as its lower triangle (D[a][c], a >= c; the upper
// entries are read through the symmetry).  All global stores come after the
// last workgroup barrier, so no barrier waits for them.  Global loads and
// stores run with consecutive threads on consecutive rows of a band column.
__device__ void bulge_step(double* __restrict__ AB, int64_t ldab, int64_t n, int b,
                           double* __restrict__ V2, double* __restrict__ tau2, int64_t i,
                           int64_t k, BulgeSmem& sm) {
  double (*O)[kBand + 1] = sm.O;
  double (*D)[kBand + 1] = sm.D;
  double *v = sm.v, *vp = sm.vp, *y = sm.y, *z = sm.z, *x = sm.x, *yo = sm.yo, *sc = sm.sc;
  const int tid = threadIdx.x;
  const int q = tid & 3, rr = tid >> 2;  // 4 lanes per row (or column) rr
  const int64_t r0 = i + 1 + k * b;
  const int64_t r1 = min(i + (k + 1) * b, n - 1);
  const int L = (int)(r1 - r0 + 1);
  const int64_t p0 = i + 1 + (k - 1) * b;  // previous window (k >= 1; always b long)
  const int64_t f = sweep_first_step(n, b, i);

  // ---- loads (all issued before any LDS store) ----
  constexpr int EPT = kBand * kBand / 256;  // elements per thread
  {
    double dv[EPT], ov[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int c = e / kBand, a = e - c * kBand;
      dv[u] = (a >= c && a < L) ? AB[(r0 + c) * ldab + (a - c)] : 0.0;
      ov[u] = (k > 0 && a < L && c < b) ? AB[(p0 + c) * ldab + (b + a - c)] : 0.0;
    }
    double xv = 0.0;
    if (tid < kBand) {
      if (k == 0)
        xv = tid < L ? AB[i * ldab + 1 + tid] : 0.0;
      else
        xv = tid < b ? V2[(f + k - 1) * b + tid] : 0.0;
    }
    const double tp = (k > 0 && tid == 0) ? tau2[f + k - 1] : 0.0;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int c = e / kBand, a = e - c * kBand;
      if (a >= c) D[a][c] = dv[u];
      O[a][c] = ov[u];
    }
    if (tid < kBand) {
      if (k == 0)
        x[tid] = xv;
      else
        vp[tid] = xv;
    }
    if (k > 0 && tid == 0) sc[3] = tp;
  }
  __syncthreads();
  const double taup = k > 0 ? sc[3] : 0.0;
  if (k > 0) {
    // O' = O (I - taup vp vp^T) = O - taup yo vp^T (yo = O vp) is never formed: its first
    // column is the vector to annihilate, and the stores below apply both reflectors
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kBand / 4; ++u) s += O[rr][q + 4 * u] * vp[q + 4 * u];
    s = quad_sum(s);
    if (q == 0) yo[rr] = s;
    __syncthreads();
    // (wave 0 writes x and reduces it in householder: no barrier in between)
    if (tid < kBand) x[tid] = O[tid][0] - taup * yo[tid] * vp[0];
  }
  householder(x, L, v, sc);  // v, sc[0] = tau, sc[1] = beta
  const double tau = sc[0], beta = sc[1];
  if (k > 0) {
    // O^T v; the bulge becomes H O' = O' - tau v z^T with z = O'^T v = O^T v - taup vp (yo . v)
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kBand / 4; ++u) s += v[q + 4 * u] * O[q + 4 * u][rr];
    s = quad_sum(s);
    if (q == 0) z[rr] = s;
  }
  // diagonal block D <- H D H = D - v w^T - w v^T, w = y - 1/2 tau (y . v) v, y = tau D v
  {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kBand / 4; ++u) {
      const int c = q + 4 * u;
      s += (c <= rr ? D[rr][c] : D[c][rr]) * v[c];
    }
    s = quad_sum(s);
    if (q == 0) y[rr] = tau * s;
  }
  __syncthreads();
  if (tid < 64) {
    const double wv = wave_sum(y[tid] * v[tid]);
    const double yv = k > 0 ? wave_sum(yo[tid] * v[tid]) : 0.0;
    if (tid == 0) {
      sc[2] = -0.5 * tau * wv;
      sc[4] = yv;
    }
  }
  __syncthreads();
  const double al = sc[2], yov = sc[4];
  // ---- stores ----
  if (k == 0) {
    if (tid < L) AB[i * ldab + 1 + tid] = tid == 0 ? beta : 0.0;
  } else {
    // first column -> beta e_1, the other columns <- H O (all values first, then the stores)
    double ov[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int c = e / kBand, a = e - c * kBand;
      const double op = O[a][c] - taup * yo[a] * vp[c];  // O'
      ov[u] = c == 0 ? (a == 0 ? beta : 0.0) : op - tau * v[a] * (z[c] - taup * vp[c] * yov);
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int c = e / kBand, a = e - c * kBand;
      if (a < L && c < b) AB[(p0 + c) * ldab + (b + a - c)] = ov[u];
    }
  }
  {
    double dv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int c = e / kBand, a = e - c * kBand;
      const double wa = y[a] + al * v[a], wc = y[c] + al * v[c];
      dv[u] = c <= a ? D[a][c] - v[a] * wc - wa * v[c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int c = e / kBand, a = e - c * kBand;
      if (a < L && c <= a) AB[(r0 + c) * ldab + (a - c)] = dv[u];
    }
  }
  if (tid < b) V2[(f + k) * b + tid] = v[tid];
  if (tid == 0) tau2[f + k] = tau;
}

// Bulge-chasing schedule: step k of sweep i runs at time kLag i + k.  Step
// (i, k) reads and writes the band entries with rows in its window
// [i + 1 + k b, i + (k + 1) b] (the previous window's columns for k > 0), so
// the step (i + 1, k - 2) of the same time ends its rows before that window
// starts, and every entry shared by two steps is reached by the lower sweep
// first: with lag 2 the steps of one time are independent and the order of
// the sequential reduction is kept (checked on the CPU entry by entry).
constexpr int64_t kLag = 2;

// Step k = t - kLag i of every sweep i of time t, one workgroup each (one launch per time).
__global__ __launch_bounds__(256) void k_bulge(double* __restrict__ AB, int64_t ldab, int64_t n,
                                               int b, double* __restrict__ V2,
                                               double* __restrict__ tau2, int64_t t,
                                               int64_t i_lo) {
  const int64_t i = i_lo + blockIdx.x;
  const int64_t k = t - kLag * i;
  if (i > n - 3 || k < 0) return;
  const int64_t K = (n - 1 - i + b - 1) / b;
  if (k >= K) return;
  __shared__ BulgeSmem sm;
  bulge_step(AB, ldab, n, b, V2, tau2, i, k, sm);
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
// a group of `spg` consecutive slabs of kSlabW columns of X ([n][ncols]
// column-major, ld n):
//   TRANS false: B = I - V T V^T   (the block's reflectors from its highest
//                sweep down; anti-diagonals in ascending order give X <- Q2 X);
//   TRANS true:  B = I - V T^T V^T (lowest sweep first; anti-diagonals in
//                descending order give X <- Q2^T X).
// The block touches rows [J g + 1 + k b, J g + g - 1 + (k + 1) b] of X.  V
// (generated from the compact reflector rows, zero outside a reflector's b
// rows) and T are staged in LDS once per workgroup; the slabs then go through
// one at a time, the next slab's rows loading into registers while the
// current one is multiplied.  The three products W = V^T X_b, W2 = T W (or
// T^T W) and X_b -= V W2 run on the FP64 matrix cores (v_mfma_f64_16x16x4:
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16], accumulator element
// q is D[4 q + l / 16][l % 16]).
constexpr int kSlabW = 32;
constexpr int kRows = 2 * kBand;  // b + g - 1 rows, padded
constexpr int kSlabPre = kSlabW * kRows / 256;  // slab elements per thread
constexpr int64_t kQ2Wgs = 1024;  // workgroups a band back-transformation launch aims for
typedef double f64x4_t __attribute__((ext_vector_type(4)));
template <bool TRANS>
__global__ __launch_bounds__(256, 2) void k_q2_apply(double* __restrict__ X, int64_t n,
                                                     int64_t ncols, int b,
                                                     const double* __restrict__ V2,
                                                     const int64_t* __restrict__ off,
                                                     const double* __restrict__ Tb,
                                                     const int64_t* __restrict__ boff, int64_t t,
                                                     int64_t nJ, int64_t J_lo, int64_t ngrp,
                                                     int64_t spg) {
  const int64_t jj = blockIdx.x / ngrp, grp = blockIdx.x - jj * ngrp;
  const int64_t J = J_lo + jj;
  const int64_t k = t - (nJ - 1 - J);
  if (J >= nJ || k < 0) return;
  const int g = b;
  const int64_t c_lo = J * g;
  const int64_t c_hi = min(c_lo + g, n - 2) - 1;
  if (c_hi < c_lo || k >= (n - 1 - c_lo + b - 1) / b) return;
  const int64_t nslab = (ncols + kSlabW - 1) / kSlabW;
  const int64_t s0 = grp * spg;
  const int64_t s1 = min(s0 + spg, nslab);
  if (s0 >= s1) return;
  __shared__ double Xb[kRows][kSlabW + 1];
  __shared__ double W[kBand][kSlabW + 1];
  const int tid = threadIdx.x;
  const int64_t R0 = c_lo + 1 + k * b;
  const int64_t R1 = min(c_hi + (k + 1) * b, n - 1);
  const int NR = (int)(R1 - R0 + 1);
  const double* Tg = Tb + (boff[J] + k) * (kBand * kBand);
  // slab element i of this thread: column cl = (tid + 256 i) / kRows, row
  // r = tid % kRows (consecutive threads on consecutive rows); rows past the
  // block and columns past X load a clamped, valid element and are stored to
  // LDS as zeros, so the loads of a slab need no wait before the next use.
  const int r_t = tid % kRows;
  const int cl_t = tid / kRows;
  const int64_t r_ld = R0 + (r_t < NR ? r_t : NR - 1);
  double pre[kSlabPre];
  auto gload = [&](int64_t col0, int ncol) {
#pragma unroll
    for (int i = 0; i < kSlabPre; ++i) {
      const int cl = cl_t + i * (256 / kRows);
      pre[i] = X[(col0 + (cl < ncol ? cl : ncol - 1)) * n + r_ld];
    }
  };
  auto ncol_of = [&](int64_t sl) { return (int)min((int64_t)kSlabW, ncols - sl * kSlabW); };
  gload(s0 * kSlabW, ncol_of(s0));
  const int lane = tid & 63, w = tid >> 6;
  const int lm = lane & 15, lk = lane >> 4;
  // The block's V and T entries each lane's matrix-core operands need, kept in
  // registers for all slabs (gathered once; LDS holds only the slab and W, so
  // two workgroups share a compute unit).  V(r, o): entry a = r - o of
  // reflector o (zero outside 0 <= a < b, or where the reflector is missing).
  auto vget = [&](int r, int o) -> double {
    const int a = r - o;
    const int64_t c = c_lo + o;
    if (a < 0 || a >= kBand || c > c_hi || k >= (n - 1 - c + b - 1) / b) return 0.0;
    return V2[(off[c] + k) * b + a];
  };
  double v1[20], t2[kBand / 4], v3[kBand / 4][2];
#pragma unroll
  for (int u = 0; u < 20; ++u) v1[u] = vget(16 * w + 4 * u + lk, 16 * w + lm);
#pragma unroll
  for (int ks = 0; ks < kBand / 4; ++ks) {
    const int i = 16 * w + lm, j = 4 * ks + lk;
    t2[ks] = TRANS ? Tg[j * kBand + i] : Tg[i * kBand + j];
#pragma unroll
    for (int u = 0; u < 2; ++u) v3[ks][u] = vget(16 * (2 * w + u) + lm, 4 * ks + lk);
  }
  for (int64_t sl = s0; sl < s1; ++sl) {
    const int64_t col0 = sl * kSlabW;
    const int ncol = ncol_of(sl);
    __syncthreads();  // the previous slab's write-out is done with Xb
#pragma unroll
    for (int i = 0; i < kSlabPre; ++i) {
      const int cl = cl_t + i * (256 / kRows);
      Xb[r_t][cl] = (cl < ncol && r_t < NR) ? pre[i] : 0.0;
    }
    __syncthreads();
    if (sl + 1 < s1) gload(col0 + kSlabW, ncol_of(sl + 1));
    // W = V^T X_b: wave w owns rows o of tile w, both column tiles; k = r over
    // the 80 rows that reflectors 16w .. 16w + 15 reach (r = 16w .. 16w + 79;
    // the trip counts of all three products are fixed, so the loops unroll
    // and the LDS reads run ahead of the matrix-core instructions)
    {
      f64x4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 20; ++u) {
        const int r = 16 * w + 4 * u + lk;
        const double av = v1[u];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Xb[r][lm], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Xb[r][16 + lm], acc1, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        W[16 * w + 4 * q + lk][lm] = acc0[q];
        W[16 * w + 4 * q + lk][16 + lm] = acc1[q];
      }
    }
    __syncthreads();
    // W2 = T W or T^T W (T upper triangular, stored with its zeros), back into W
    {
      f64x4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < kBand / 4; ++ks) {
        const int j = 4 * ks + lk;
        const double av = t2[ks];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, W[j][lm], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, W[j][16 + lm], acc1, 0, 0, 0);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        W[16 * w + 4 * q + lk][lm] = acc0[q];
        W[16 * w + 4 * q + lk][16 + lm] = acc1[q];
      }
    }
    __syncthreads();
    // X_b -= V W2: wave w owns row tiles 2w, 2w + 1, both column tiles; k = o
    {
      f64x4_t acc[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < kBand / 4; ++ks) {
        const int o = 4 * ks + lk;
        const double b0 = W[o][lm], b1 = W[o][16 + lm];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double av = v3[ks][u];
          acc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[u][0], 0, 0, 0);
          acc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[u][1], 0, 0, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * (2 * w + u) + 4 * q + lk;
          Xb[r][lm] -= acc[u][0][q];
          Xb[r][16 + lm] -= acc[u][1][q];
        }
    }
    __syncthreads();
    for (int e = tid; e < kSlabW * kRows; e += 256) {
      const int c2 = e / kRows, r = e - c2 * kRows;
      if (c2 < ncol && r < NR) X[(col0 + c2) * n + R0 + r] = Xb[r][c2];
    }
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
// tridiagonal matrix (column-major) and evals the eigenvalues, ascending.  With
// stage3 false the tridiagonal matrix is left in the W_EIG_DE slot (d, then e)
// instead.
// Panels whose two-sided update of the trailing matrix is delayed and applied
// as one product (k = 2 b kDelay).
constexpr int kDelay = 8;

static int ts_reduce(qsgw_ctx* c, int64_t n, double* A, double* evals, const char* what,
                     TwoStage* ts, bool stage3 = true) {
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
  CHECK(ws_get(c, W_EIG_U, (size_t)(4 * kDelay * n * b), &U1));  // 2 x [n][2 b kDelay]
  U2 = nullptr;
  CHECK(ws_get(c, W_EIG_XY, (size_t)(2 * n * b + 2 * b * b + 2 * kDelay * b * b), &X));
  Y = X + n * b;
  Z1 = Y + n * b;
  Z2 = Z1 + b * b;
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  // The two-sided update of the trailing matrix, S <- S - U1 U2^T with
  // U1 = [V W], U2 = [W V], is delayed over up to kDelay panels: the pending
  // blocks sit side by side in U1a, U2a ([n][2 b kDelay], row r of the matrix
  // at row r), the next panel's columns and its product X = S Y are corrected
  // with them (two thin products), and the stored matrix takes all of them in
  // one product with k = 2 b (pending panels).
  double* U1a = U1;
  double* U2a = U1 + 2 * kDelay * n * b;
  int dp = 0;  // pending panels
  // cooperative panel QR: barrier flags (cleared for this solve) and error flag
  unsigned long long* pflags = nullptr;
  int* perr = nullptr;
  if (c->tiles.panel_coop) {
    CHECK(ws_get(c, W_EIG_PFLAG, 257, &pflags));
    perr = reinterpret_cast<int*>(pflags + 256);
    HIP_TRY(c, hipMemsetAsync(pflags, 0, 257 * sizeof(unsigned long long), c->stream));
  }
  for (int64_t p = 0; p < np; ++p) {
    const int64_t j = ts->pj[p], m = ts->pm[p], kk = m < b ? m : b;
    const int mi = (int)m;
    double* P = A + j * n + (j + b);
    double* S = A + (j + b) * n + (j + b);
    double* V = V1 + ts->poff[p];
    double* T = T1 + p * b * b;
    const int64_t Kp = 2 * b * dp;  // k of the pending blocks
    if (dp > 0) {
      // columns j .. j+b-1, rows j .. n-1: A -= U1a U2a^T (the panel and the diagonal block)
      Strided<false> A2{U2a + j, 1, n, 0, b};
      Strided<false> B1{U1a + j, 1, n, 0, n - j};
      EpiSub E{A + j * n + j, n};
      CHECK((gemm_shape<double, false>(c, SH_64x64, "eig/sy2sb panel", A2, B1, E, b, n - j, Kp,
                                       1)));
    }
    bool coop_done = false;
    if (m >= 2 * b && pflags && (m + 255) / 256 <= 256) {
      // the whole panel in one cooperative launch (see k_panel_coop; one flag per workgroup)
      const int G = (int)((m + 255) / 256);
      double *part, *Rbuf;
      CHECK(ws_get(c, W_EIG_PANEL, (size_t)(2 * G * b + 2 * b + b * b), &part));
      double* rowj = part + 2 * G * b;
      Rbuf = rowj + 2 * b;
      int64_t lda = n, mm = m;
      double* tp = tau1 + p * b;
      unsigned long long gen0 = (unsigned long long)p * (unsigned long long)b;
      void* args[] = {&P, &lda, &mm, &part, &rowj, (void*)&G, &Rbuf, &tp, &pflags, &gen0, &perr};
      const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_panel_coop),
                                                      dim3((unsigned)G), dim3(256), args, 0,
                                                      c->stream);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_panel_r, dim3(blocks_for(b * b)), dim3(256), 0, c->stream, P, n, b,
                           Rbuf);
        CHECK(launch_check(c, "k_panel_coop"));
        coop_done = true;
      } else {
        // not resident at once on this device: the per-column launches below
        (void)hipGetLastError();
      }
    }
    if (coop_done) {
    } else if (m >= 2 * b) {
      // one launch per column (see k_panel_col)
      const int rpt = m > 16384 ? 2 : 1;  // rows per thread
      const int G = (int)((m + 256 * rpt - 1) / (256 * rpt));
      double *part, *Rbuf;
      CHECK(ws_get(c, W_EIG_PANEL, (size_t)(2 * G * b + b * b), &part));
      Rbuf = part + 2 * G * b;
      for (int jc = -1; jc < b; ++jc) {
        double* pin = part + (size_t)((jc + 2) & 1) * G * b;
        double* pout = part + (size_t)((jc + 1) & 1) * G * b;
        if (rpt == 2)
          hipLaunchKernelGGL(k_panel_col<2>, dim3((unsigned)G), dim3(256), 0, c->stream, P, n, m, b,
                             jc, pin, pout, G, Rbuf, tau1 + p * b);
        else
          hipLaunchKernelGGL(k_panel_col<1>, dim3((unsigned)G), dim3(256), 0, c->stream, P, n, m, b,
                             jc, pin, pout, G, Rbuf, tau1 + p * b);
      }
      hipLaunchKernelGGL(k_panel_r, dim3(blocks_for(b * b)), dim3(256), 0, c->stream, P, n, b, Rbuf);
      CHECK(launch_check(c, "k_panel_col"));
    } else {
      RB_TRY(c, rocsolver_dgeqrf(h, mi, b, P, ni, tau1 + p * b), what);
    }
    // this panel's block of the pending operands: columns [2 b dp, 2 b (dp + 1))
    double* U1s = U1a + 2 * b * dp * n + (j + b);
    double* U2s = U2a + 2 * b * dp * n + (j + b);
    if (kk < b) {
      HIP_TRY(c, hipMemset2DAsync(U1s, n * sizeof(double), 0, m * sizeof(double), 2 * b, c->stream));
      HIP_TRY(c, hipMemset2DAsync(U2s, n * sizeof(double), 0, m * sizeof(double), 2 * b, c->stream));
    }
    hipLaunchKernelGGL(k_panel_v, dim3(blocks_for(m * kk)), dim3(256), 0, c->stream, P, n, m, kk,
                       V, U1s, U2s + b * n, n);
    CHECK(launch_check(c, "k_panel_v"));
    // T from the reflectors' Gram matrix (V^T V, long k = m) and tau
    {
      Strided<true> Av{V, m, 1, 0, kk};
      CHECK(gemm_long_k(c, "eig/sy2sb gram", Av, Av, Z1, kk, kk, m));
      hipLaunchKernelGGL(k_panel_t, dim3(1), dim3(256), 0, c->stream, Z1, (int)kk, tau1 + p * b, T,
                         b);
      CHECK(launch_check(c, "k_panel_t"));
    }
    // Y = V T  (Y^T[c][r] = sum_l T(l, c) V(r, l))
    {
      Strided<true> At{T, b, 1, 0, kk};
      Strided<false> Bv{V, 1, m, 0, m};
      EpiStore E{Y, m, 0, 0, 1.0};
      CHECK((gemm_shape<double, false>(c, SH_64x64, "eig/sy2sb Y", At, Bv, E, kk, m, kk, 1)));
    }
    // X = S Y  (X^T[c][r] = sum_k Y[k][c] S[k][r], S symmetric), split over k,
    // minus the pending updates: X -= U1a (U2a^T Y) on rows j+b .. n-1
    {
      Strided<true> Ay{Y, m, 1, 0, kk};
      Strided<true> Bs{S, n, 1, 0, m};
      CHECK(gemm_long_k(c, "eig/sy2sb X", Ay, Bs, X, kk, m, m));
      if (dp > 0) {
        double* Gp = Z2 + b * b;  // [Kp][kk]
        Strided<true> Au{U2a + j + b, n, 1, 0, Kp};
        CHECK(gemm_long_k(c, "eig/sy2sb X corr", Au, Ay, Gp, Kp, kk, m));
        Strided<false> Ag{Gp, 1, kk, 0, kk};
        Strided<false> Bu{U1a + j + b, 1, n, 0, m};
        EpiSub E{X, m};
        CHECK((gemm_shape<double, false>(c, SH_64x64, "eig/sy2sb X corr", Ag, Bu, E, kk, m, Kp, 1)));
      }
    }
    // Z1 = V^T X  (Z1[i][c] = sum_r V(r, i) X(r, c)), Z2 = T^T Z1
    {
      Strided<true> Av{V, m, 1, 0, kk};
      Strided<true> Bx{X, m, 1, 0, kk};
      CHECK(gemm_long_k(c, "eig/sy2sb Z1", Av, Bx, Z1, kk, kk, m));
      Strided<true> At{T, b, 1, 0, kk};
      Strided<false> Bz{Z1, 1, kk, 0, kk};
      EpiStore E{Z2, kk, 0, 0, 1.0};
      CHECK((gemm_shape<double, false>(c, SH_64x64, "eig/sy2sb Z2", At, Bz, E, kk, kk, kk, 1)));
    }
    // W = X - 1/2 V Z2 into this panel's W halves of U1a and U2a
    {
      Strided<false> Az{Z2, 1, kk, 0, kk};
      Strided<false> Bv{V, 1, m, 0, m};
      EpiPanelW E{X, U1s + b * n, U2s, m, n};
      CHECK((gemm_shape<double, false>(c, SH_64x64, "eig/sy2sb W", Az, Bv, E, kk, m, kk, 1)));
    }
    ++dp;
    if (dp == kDelay || p == np - 1) {
      // S -= U1a U2a^T: the sum of the pending V W^T + W V^T is symmetric, so
      // only the upper tiles are computed and each is written to both halves
      Strided<false> A2{U2a + j + b, 1, n, 0, m};
      Strided<false> B1{U1a + j + b, 1, n, 0, m};
      EpiSubSym E{S, n, m};
      CHECK((gemm_shape<double, true>(c, SH_128x128, "eig/sy2sb update", A2, B1, E, m, m,
                                      2 * b * dp, 1)));
      dp = 0;
    }
  }

  if (perr) {
    int stalled = 0;
    CHECK(read_flag(c, perr, &stalled));
    if (stalled) return fail(c, QSGW_ERR_SOLVER, "%s: panel QR barrier wait exceeded its bound", what);
  }

  // ---- stage 2: band -> tridiagonal ----
  const int64_t ldab = 2 * b + 1;
  std::vector<int64_t> hoff((size_t)n, 0);
  int64_t nref = 0, tmax = 0;
  for (int64_t i = 0; i <= n - 3; ++i) {
    if (sweep_first_step(n, b, i) != nref)
      return fail(c, QSGW_ERR_SOLVER, "%s: bulge step offset of sweep %lld", what, (long long)i);
    hoff[(size_t)i] = nref;
    const int64_t K = (n - 1 - i + b - 1) / b;
    nref += K;
    if (kLag * i + K > tmax) tmax = kLag * i + K;
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
    int64_t i_hi = t / kLag;
    if (i_hi > n - 3) i_hi = n - 3;
    int64_t i_lo = t - K0 >= 0 ? (t - K0) / kLag + 1 : 0;  // kLag i > t - K0
    if (i_lo > i_hi) continue;
    hipLaunchKernelGGL(k_bulge, dim3((unsigned)(i_hi - i_lo + 1)), dim3(256), 0, c->stream, AB,
                       ldab, n, b, V2, tau2, t, i_lo);
  }
  CHECK(launch_check(c, "k_bulge"));
  hipLaunchKernelGGL(k_tridiag, dim3(blocks_for(n)), dim3(256), 0, c->stream, AB, n, ldab, dd, ee);
  CHECK(launch_check(c, "k_tridiag"));
  hipLaunchKernelGGL(k_q2_tfactor, dim3((unsigned)nJ, (unsigned)K0), dim3(256), 0, c->stream, V2,
                     tau2, off, off + n, n, b, ts->Tb);
  CHECK(launch_check(c, "k_q2_tfactor"));

  if (!stage3) return QSGW_OK;
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
    // slabs per workgroup: as many as keep at least kQ2Wgs workgroups in the launch
    // (the block's V and T are staged once per workgroup)
    const int64_t nb = J_hi - J_lo + 1;
    int64_t ngrp = (kQ2Wgs + nb - 1) / nb;
    if (ngrp > nslab) ngrp = nslab;
    const int64_t spg = (nslab + ngrp - 1) / ngrp;
    ngrp = (nslab + spg - 1) / spg;
    if (trans)
      hipLaunchKernelGGL(k_q2_apply<true>, dim3((unsigned)(nb * ngrp)), dim3(256), 0, c->stream, X,
                         n, ncols, b, ts.V2, ts.off, ts.Tb, ts.off + n, t, ts.nJ, J_lo, ngrp, spg);
    else
      hipLaunchKernelGGL(k_q2_apply<false>, dim3((unsigned)(nb * ngrp)), dim3(256), 0, c->stream,
                         X, n, ncols, b, ts.V2, ts.off, ts.Tb, ts.off + n, t, ts.nJ, J_lo, ngrp,
                         spg);
  };
  double *W1 = nullptr, *W2 = nullptr, *WP = nullptr;
  CHECK(ws_get(c, W_EIG_Q1W, (size_t)(2 * b * ncols), &W1));
  W2 = W1 + b * ncols;
  // X[j+b:, :] <- (I - V T V^T) X (trans false) or (I - V T^T V^T) X (trans true),
  // as W1 = V^T X (split over the long k = rows), W2 = T W1 or T^T W1, X -= V W2
  auto q1 = [&](int64_t p) -> int {
    const int64_t j = ts.pj[(size_t)p], m = ts.pm[(size_t)p], kk = m < b ? m : b;
    const double* V = ts.V1 + ts.poff[(size_t)p];
    double* Xs = X + (j + b);
    {
      Strided<true> Av{V, m, 1, 0, kk};
      Strided<true> Bx{Xs, n, 1, 0, ncols};
      const int64_t tiles = ((kk + 63) / 64) * ((ncols + 63) / 64);
      const SplitPlan sp = round_chunks(split_plan(m, splits_for(tiles, m, 2048)), m, 32);
      if (sp.nz > 1) {
        CHECK(ws_get(c, W_EIG_XP, (size_t)(sp.nz * kk * ncols), &WP));
        EpiStore E{WP, ncols, 0, kk * ncols, 1.0};
        CHECK((gemm_shape<double, false, 32>(c, SH_64x64, "eig/q1 W", Av, Bx, E, kk, ncols, m, 1,
                                             sp)));
        hipLaunchKernelGGL(k_sum_slices, dim3(blocks_for(kk * ncols)), dim3(256), 0, c->stream, WP,
                           sp.nz, kk * ncols, sp.nz, W1);
        CHECK(launch_check(c, "k_sum_slices"));
      } else {
        EpiStore E{W1, ncols, 0, 0, 1.0};
        CHECK((gemm_shape<double, false, 32>(c, SH_64x64, "eig/q1 W", Av, Bx, E, kk, ncols, m, 1)));
      }
    }
    {
      // W2[i][c] = sum_l T(i, l) W1[l][c] (or T(l, i)): the row-major kk x ncols W1, W2 are
      // column-major ncols x kk for rocBLAS, so W2^T = W1^T T^T (or W1^T T)
      const double one = 1.0, zero = 0.0;
      RB_TRY(c, rocblas_dgemm(c->blas, rocblas_operation_none,
                              trans ? rocblas_operation_none : rocblas_operation_transpose, nc,
                              (int)kk, (int)kk, &one, W1, nc, ts.T1 + p * b * b, b, &zero, W2, nc),
             what);
    }
    {
      // X^T[c][r] -= sum_i W2[i][c] V[r][i]
      Strided<false> Aw{W2, 1, ncols, 0, ncols};
      Strided<false> Bv{V, 1, m, 0, m};
      EpiSub E{Xs, n};
      CHECK((gemm_shape<double, false>(c, SH_128x128, "eig/q1 update", Aw, Bv, E, ncols, m, kk,
                                       1)));
    }
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
//   R^T = E^T (Q2^T Q1^T Bt^T),
// and E^T is applied by the tridiagonal merge (tridiag_project_dc), which
// never forms E either.  A is destroyed; X: [naux][n] work array.
int eig_two_stage_project(qsgw_ctx* c, int64_t n, double* A, double* evals, int64_t naux,
                          const double* Bt, double* X, double* R, const char* what) {
  if (n > 46340) return fail(c, QSGW_ERR_UNSUPPORTED, "%s: n too large for the two-stage solver", what);
  if (naux > 0x7fffffffLL) return fail(c, QSGW_ERR_UNSUPPORTED, "%s: naux too large", what);
  if (n < 4 * kBand) {
    CHECK(syevd(c, n, A, evals, what));  // A = Z
    const double one = 1.0, zero = 0.0;
    RB_TRY(c, rocblas_dgemm(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)n,
                            (int)naux, (int)n, &one, A, (int)n, Bt, (int)n, &zero, R, (int)n),
           what);
    return QSGW_OK;
  }
  TwoStage ts;
  CHECK(ts_reduce(c, n, A, evals, what, &ts, false));
  HIP_TRY(c, hipMemcpyAsync(X, Bt, (size_t)(naux * n) * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
  CHECK(ts_apply(c, ts, n, X, naux, true, what));
  double* dd = nullptr;
  CHECK(ws_get(c, W_EIG_DE, (size_t)(2 * n), &dd));
  return tridiag_project_dc(c, n, dd, dd + n, A, naux, X, evals, R, what);
}
