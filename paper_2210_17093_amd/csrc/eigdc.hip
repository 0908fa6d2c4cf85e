// Tridiagonal stage of the two-stage Casida eigensolver in projection mode:
// the top divide-and-conquer merge is done here, the two halves by rocSOLVER.
//
// The tridiagonal T (order n, diagonal d, off-diagonal e) is torn at
// n1 = n / 2 (Cuppen): with beta = e[n1 - 1],
//   T = diag(T1, T2) + |beta| v v^T,  v = e_{n1-1} + sign(beta) e_{n1},
// where T1 and T2 are the leading and trailing blocks with |beta| taken off
// their touching diagonal entries.  With T1 = E1 D1 E1^T and T2 = E2 D2 E2^T
// (rocSOLVER dstedc) and Q = diag(E1, E2), T = Q (D + rho z z^T) Q^T with
// z = Q^T v / |Q^T v| and rho = |beta| |Q^T v|^2.  The eigenpairs of the
// rank-one modification D + rho z z^T (poles d sorted ascending):
//   - deflated: a pole with rho |z_i| <= tol = 8 eps max(max |d|, rho) is an
//     eigenvalue with its unit vector; of two neighbouring poles i < j whose
//     rotation zeroing z_i leaves an off-diagonal |c s (d_j - d_i)| <= tol, the
//     rotated pole i is one (with value c^2 d_i + s^2 d_j);
//   - the K others: the roots lambda_j of the secular equation
//     f(lambda) = 1 + rho sum_i z_i^2 / (d_i - lambda) = 0, one in each
//     (d_j, d_{j+1}) and the last in (d_K, d_K + rho), with eigenvectors
//     u_j ~ zh / (d - lambda_j), where zh is recomputed from the roots,
//     zh_i^2 = prod_j (lambda_j - d_i) / (rho prod_{j != i} (d_j - d_i))
//     (the Gu-Eisenstat form, which keeps the u_j orthogonal to working
//     precision).  Each root is found relative to its nearer pole o
//     (lambda = d_o + mu, every d_i - lambda formed as (d_i - d_o) - mu), by
//     Newton steps on h(mu) = mu f(mu), which has no pole at mu = 0, kept
//     inside a bisection bracket.
// Projection mode needs R = E^T X only (E the eigenvectors of T, X an
// n x naux matrix), so E is never formed: R = U^T (Q^T X) with the rows of
// Q^T X sorted, rotated and split into deflated rows (copied to their
// columns of R) and the K others (one product with U).  Everything in FP64.
#include "internal.hpp"

namespace {

__device__ __forceinline__ double dc_wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ double dc_wave_prod(double x) {
  for (int o = 32; o > 0; o >>= 1) x *= __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ double dc_wave_max(double x) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  return x;
}

// Number of entries of the ascending v[0..len) below x (strict: < x) or not
// above it (<= x).
__device__ __forceinline__ int64_t count_below(const double* v, int64_t len, double x,
                                               bool or_equal) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const bool below = or_equal ? v[mid] <= x : v[mid] < x;
    if (below) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Tear T at n1: scal[0] = beta = e[n1 - 1]; |beta| off d[n1 - 1] and d[n1].
__global__ void k_dc_tear(double* __restrict__ d, const double* __restrict__ e, int64_t n1,
                          double* __restrict__ scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double beta = e[n1 - 1];
  scal[0] = beta;
  d[n1 - 1] -= fabs(beta);
  d[n1] -= fabs(beta);
}

// The halves' eigenvalues (w1 = d[0..n1), w2 = d[n1..n), each ascending) merged
// into ds ascending (ties: the first half first), with z (unnormalised: row
// n1 - 1 of E1, sign(beta) times row 0 of E2) and the source row of Q^T X.
__global__ void k_dc_prep(const double* __restrict__ d, int64_t n1, int64_t n2,
                          const double* __restrict__ E1, const double* __restrict__ E2,
                          const double* __restrict__ scal, double* __restrict__ ds,
                          double* __restrict__ zs, int64_t* __restrict__ src) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n1 + n2) return;
  const double sg = scal[0] < 0.0 ? -1.0 : 1.0;
  int64_t pos;
  double v, z;
  if (t < n1) {
    v = d[t];
    pos = t + count_below(d + n1, n2, v, false);
    z = E1[t * n1 + (n1 - 1)];
  } else {
    const int64_t t2 = t - n1;
    v = d[n1 + t2];
    pos = t2 + count_below(d, n1, v, true);
    z = sg * E2[t2 * n2];
  }
  ds[pos] = v;
  zs[pos] = z;
  src[pos] = t;
}

// Gs[s][P] = G[src[s]][P] (rows of naux values).
__global__ void k_dc_gather_rows(const double* __restrict__ G, const int64_t* __restrict__ src,
                                 int64_t n, int64_t naux, double* __restrict__ Gs) {
  const int64_t s = blockIdx.y;
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n || P >= naux) return;
  Gs[s * naux + P] = G[src[s] * naux + P];
}

// Deflation, one workgroup.  z is normalised in place, rho = |beta| |z|^2 and
// tol go to scal[1], scal[2]; then thread 0 walks the poles in order (staged
// through LDS in chunks) and emits the non-deflated poles (nd, dk, zk), the
// deflated ones (df, dfv) and the rotations (ra, rb, rc, rs) in the order
// they are to be applied.  cnt = {K, deflated, rotations}.
constexpr int kDcChunk = 2048;
__global__ __launch_bounds__(256) void k_dc_deflate(const double* __restrict__ ds,
                                                    double* __restrict__ zs, int64_t n,
                                                    double* __restrict__ scal,
                                                    int64_t* __restrict__ nd,
                                                    double* __restrict__ dk,
                                                    double* __restrict__ zk,
                                                    int64_t* __restrict__ df,
                                                    double* __restrict__ dfv,
                                                    int64_t* __restrict__ ra,
                                                    int64_t* __restrict__ rb,
                                                    double* __restrict__ rc,
                                                    double* __restrict__ rs,
                                                    int64_t* __restrict__ cnt) {
  __shared__ double red[2][4];
  __shared__ double dl[kDcChunk], zl[kDcChunk];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double s2 = 0.0, dm = 0.0;
  for (int64_t i = tid; i < n; i += 256) {
    s2 += zs[i] * zs[i];
    dm = fmax(dm, fabs(ds[i]));
  }
  s2 = dc_wave_sum(s2);
  dm = dc_wave_max(dm);
  if (lane == 0) {
    red[0][w] = s2;
    red[1][w] = dm;
  }
  __syncthreads();
  s2 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  dm = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
  const double zn = sqrt(s2);
  const double rho = fabs(scal[0]) * s2;
  const double tol = 8.0 * __DBL_EPSILON__ * fmax(dm, rho);
  // serial state of thread 0: the pending candidate (not yet known to stay)
  int64_t K = 0, ndf = 0, nrot = 0, prev = -1;
  double dp = 0.0, zp = 0.0;
  for (int64_t c0 = 0; c0 < n; c0 += kDcChunk) {
    const int len = (int)(n - c0 < kDcChunk ? n - c0 : kDcChunk);
    __syncthreads();  // thread 0 is done with the previous chunk
    for (int i = tid; i < len; i += 256) {
      dl[i] = ds[c0 + i];
      zl[i] = zs[c0 + i] / zn;
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i < len; ++i) {
        const int64_t j = c0 + i;
        const double dj = dl[i], zj = zl[i];
        if (rho * fabs(zj) <= tol) {
          df[ndf] = j;
          dfv[ndf] = dj;
          ++ndf;
          continue;
        }
        if (prev < 0) {
          prev = j;
          dp = dj;
          zp = zj;
          continue;
        }
        const double tau = hypot(zp, zj);
        const double cc = zj / tau, ss = zp / tau;
        if (fabs((dj - dp) * cc * ss) <= tol) {
          // rows (prev, j) <- (c prev - s j, s prev + c j): z_prev -> 0, z_j -> tau
          ra[nrot] = prev;
          rb[nrot] = j;
          rc[nrot] = cc;
          rs[nrot] = ss;
          ++nrot;
          df[ndf] = prev;
          dfv[ndf] = dp * cc * cc + dj * ss * ss;
          ++ndf;
          prev = j;
          dp = dp * ss * ss + dj * cc * cc;
          zp = tau;
        } else {
          nd[K] = prev;
          dk[K] = dp;
          zk[K] = zp;
          ++K;
          prev = j;
          dp = dj;
          zp = zj;
        }
      }
    }
  }
  if (tid == 0) {
    if (prev >= 0) {
      nd[K] = prev;
      dk[K] = dp;
      zk[K] = zp;
      ++K;
    }
    cnt[0] = K;
    cnt[1] = ndf;
    cnt[2] = nrot;
    scal[1] = rho;
    scal[2] = tol;
  }
}

// The rotations, in order, on the rows of Gs (one thread per column).
__global__ void k_dc_rotate(double* __restrict__ Gs, int64_t naux, const int64_t* __restrict__ ra,
                            const int64_t* __restrict__ rb, const double* __restrict__ rc,
                            const double* __restrict__ rs, int64_t nrot) {
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= naux) return;
  for (int64_t r = 0; r < nrot; ++r) {
    double* xa = Gs + ra[r] * naux + P;
    double* xb = Gs + rb[r] * naux + P;
    const double a = *xa, b = *xb, c = rc[r], s = rs[r];
    *xa = c * a - s * b;
    *xb = s * a + c * b;
  }
}

// Root j of the secular equation, one wave each: its pole of origin (dor[j] =
// d_o), mu[j] = lambda_j - d_o and lam[j].
__global__ __launch_bounds__(256) void k_dc_secular(const double* __restrict__ dk,
                                                    const double* __restrict__ zk, int64_t K,
                                                    const double* __restrict__ scal,
                                                    double* __restrict__ dor,
                                                    double* __restrict__ mu,
                                                    double* __restrict__ lam) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= K) return;
  const double rho = scal[1];
  int64_t o;
  double a, b;
  if (j < K - 1) {
    const double half = 0.5 * (dk[j + 1] - dk[j]);
    double s = 0.0;
    for (int64_t i = lane; i < K; i += 64) s += zk[i] * zk[i] / ((dk[i] - dk[j]) - half);
    s = dc_wave_sum(s);
    if (1.0 + rho * s >= 0.0) {
      o = j;
      a = 0.0;
      b = half;
    } else {
      o = j + 1;
      a = -half;
      b = 0.0;
    }
  } else {
    o = j;
    a = 0.0;
    b = rho;
  }
  const double d_o = dk[o], z_o2 = zk[o] * zk[o];
  // f(mu) increases from -inf to +inf over the bracket: f(a) < 0 <= f(b)
  double m = 0.5 * (a + b);
  for (int it = 0; it < 256; ++it) {
    double S = 0.0, Sp = 0.0;
    for (int64_t i = lane; i < K; i += 64) {
      if (i == o) continue;
      const double dl = dk[i] - d_o;
      const double r = 1.0 / (dl - m);
      const double q = zk[i] * zk[i] * r;
      S += q;
      Sp += q * dl * r;
    }
    S = dc_wave_sum(S);
    Sp = dc_wave_sum(Sp);
    const double h = m * (1.0 + rho * S) - rho * z_o2;  // = m f(m)
    const bool fneg = m > 0.0 ? h < 0.0 : h > 0.0;
    if (fneg) a = m; else b = m;
    double mn = m - h / (1.0 + rho * Sp);
    if (!(mn > a && mn < b)) mn = 0.5 * (a + b);
    const bool done = fabs(mn - m) <= 2.0 * __DBL_EPSILON__ * fabs(mn) ||
                      !(b - a > 2.0 * __DBL_EPSILON__ * fmax(fabs(a), fabs(b)));
    m = mn;
    if (done) break;
  }
  if (lane == 0) {
    dor[j] = d_o;
    mu[j] = m;
    lam[j] = d_o + m;
  }
}

// zh_i (one wave each): the product of (lambda_j - d_i) / (d_j - d_i) over
// j < i, of (lambda_j - d_i) / (d_{j+1} - d_i) over i <= j < K - 1 (every
// factor in (0, 1) by interlacing) and (lambda_K - d_i) / rho; the sign of z_i.
__global__ __launch_bounds__(256) void k_dc_zhat(const double* __restrict__ dk,
                                                 const double* __restrict__ zk, int64_t K,
                                                 const double* __restrict__ scal,
                                                 const double* __restrict__ dor,
                                                 const double* __restrict__ mu,
                                                 double* __restrict__ zh) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= K) return;
  const double di = dk[i], rho = scal[1];
  double p = 1.0;
  for (int64_t j = lane; j < K; j += 64) {
    const double lj = (dor[j] - di) + mu[j];
    const double den = j < i ? dk[j] - di : (j < K - 1 ? dk[j + 1] - di : rho);
    p *= lj / den;
  }
  p = dc_wave_prod(p);
  if (lane == 0) zh[i] = copysign(sqrt(p), zk[i]);
}

// U[j][i] = u_j[i], the unit eigenvector of root j (one workgroup per root).
__global__ __launch_bounds__(256) void k_dc_vectors(const double* __restrict__ dk,
                                                    const double* __restrict__ zh, int64_t K,
                                                    const double* __restrict__ dor,
                                                    const double* __restrict__ mu,
                                                    double* __restrict__ U) {
  __shared__ double red[4];
  const int64_t j = blockIdx.x;
  if (j >= K) return;
  const int tid = threadIdx.x;
  const double d_o = dor[j], m = mu[j];
  double s = 0.0;
  for (int64_t i = tid; i < K; i += 256) {
    const double u = zh[i] / ((dk[i] - d_o) - m);
    s += u * u;
  }
  s = dc_wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  const double inv = 1.0 / sqrt(red[0] + red[1] + red[2] + red[3]);
  for (int64_t i = tid; i < K; i += 256) U[j * K + i] = zh[i] / ((dk[i] - d_o) - m) * inv;
}

// Deflated values in ascending order (rank by counting; ties by index):
// dfs[r], and the row of Gs each one keeps.
__global__ void k_dc_sort_deflated(const double* __restrict__ dfv, const int64_t* __restrict__ df,
                                   int64_t ndf, double* __restrict__ dfs,
                                   int64_t* __restrict__ dfrow) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ndf) return;
  const double v = dfv[q];
  int64_t r = 0;
  for (int64_t p = 0; p < ndf; ++p) {
    const double u = dfv[p];
    r += (u < v || (u == v && p < q)) ? 1 : 0;
  }
  dfs[r] = v;
  dfrow[r] = df[q];
}

// Final positions (eigenvalues ascending): root j before deflated values equal
// to it.  evals[pos] = value; posnd[j], posdf[r] for the columns of R.
__global__ void k_dc_positions(const double* __restrict__ lam, int64_t K,
                               const double* __restrict__ dfs, int64_t ndf,
                               double* __restrict__ evals, int64_t* __restrict__ posnd,
                               int64_t* __restrict__ posdf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < K) {
    const double v = lam[t];
    const int64_t p = t + count_below(dfs, ndf, v, false);
    posnd[t] = p;
    evals[p] = v;
  } else if (t < K + ndf) {
    const int64_t r = t - K;
    const double v = dfs[r];
    const int64_t p = r + count_below(lam, K, v, true);
    posdf[r] = p;
    evals[p] = v;
  }
}

// Gnd[i][P] = Gs[nd[i]][P] for the K non-deflated rows; the deflated rows
// go straight to their columns of R ([naux][n]).
__global__ void k_dc_split_rows(const double* __restrict__ Gs, const int64_t* __restrict__ nd,
                                int64_t K, const int64_t* __restrict__ dfrow,
                                const int64_t* __restrict__ posdf, int64_t ndf, int64_t naux,
                                int64_t n, double* __restrict__ Gnd, double* __restrict__ R) {
  const int64_t s = blockIdx.y;
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= naux) return;
  if (s < K) {
    Gnd[s * naux + P] = Gs[nd[s] * naux + P];
  } else if (s < K + ndf) {
    const int64_t r = s - K;
    R[P * n + posdf[r]] = Gs[dfrow[r] * naux + P];
  }
}

// R[m][pos[n]] = v: the product's columns scattered to their eigenvalue order.
struct EpiScatterCols {
  double* R;
  int64_t ld;
  const int64_t* pos;
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t m, int64_t n, double v,
                                             bool) const {
    R[m * ld + pos[n]] = v;
  }
};

}  // namespace

// Eigenvalues (ascending) of the tridiagonal T (d, e: destroyed) and
// R[P][s] = sum_r E[r][s] X[P][r] for X row-major [naux][n] (column-major
// n x naux, ld n), without forming E.  A: n x n work array.
int tridiag_project_dc(qsgw_ctx* c, int64_t n, double* d, double* e, double* A, int64_t naux,
                       const double* X, double* evals, double* R, const char* what) {
  if (n < 4) return fail(c, QSGW_ERR_INVALID_ARG, "%s: tridiagonal merge needs n >= 4", what);
  const int64_t n1 = n / 2, n2 = n - n1;
  double *G, *V, *scal;
  int64_t* I;
  int* flags;
  CHECK(ws_get(c, W_EIG_DCG, (size_t)(2 * n * naux), &G));
  CHECK(ws_get(c, W_EIG_DCV, (size_t)(12 * n + 8), &V));
  CHECK(ws_get(c, W_EIG_DCI, (size_t)(9 * n + 4), &I));
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  double* Gs = G + n * naux;
  double *ds = V, *zs = V + n, *dk = V + 2 * n, *zk = V + 3 * n, *dfv = V + 4 * n, *rc = V + 5 * n,
         *rs = V + 6 * n, *dor = V + 7 * n, *mu = V + 8 * n, *lam = V + 9 * n, *zh = V + 10 * n,
         *dfs = V + 11 * n;
  scal = V + 12 * n;
  int64_t *src = I, *nd = I + n, *df = I + 2 * n, *ra = I + 3 * n, *rb = I + 4 * n,
          *dfrow = I + 5 * n, *posnd = I + 6 * n, *posdf = I + 7 * n, *cnt = I + 9 * n;
  double* E1 = A;
  double* E2 = A + n1 * n1;
  rocblas_handle h = c->blas;

  hipLaunchKernelGGL(k_dc_tear, dim3(1), dim3(64), 0, c->stream, d, e, n1, scal);
  CHECK(launch_check(c, "k_dc_tear"));
  rocblas_status st = rocsolver_dstedc(h, rocblas_evect_tridiagonal, (rocblas_int)n1, d, e, E1,
                                       (rocblas_int)n1, (rocblas_int*)(flags + 1));
  if (st == rocblas_status_success)
    st = rocsolver_dstedc(h, rocblas_evect_tridiagonal, (rocblas_int)n2, d + n1, e + n1, E2,
                          (rocblas_int)n2, (rocblas_int*)(flags + 2));
  if (st != rocblas_status_success)
    return fail(c, QSGW_ERR_SOLVER, "%s: rocsolver_dstedc status %d", what, (int)st);
  // G = Q^T X: G[i][P] = sum_r E1[r][i] X[P][r] (first half), likewise E2 (second)
  {
    Strided<true> A1{E1, n1, 1, 0, n1};
    Strided<true> X1{X, n, 1, 0, naux};
    EpiStore S1{G, naux, 0, 0, 1.0};
    CHECK((gemm_shape<double, false>(c, SH_128x128, "eig/dc Q^T X", A1, X1, S1, n1, naux, n1, 1)));
    Strided<true> A2{E2, n2, 1, 0, n2};
    Strided<true> X2{X + n1, n, 1, 0, naux};
    EpiStore S2{G + n1 * naux, naux, 0, 0, 1.0};
    CHECK((gemm_shape<double, false>(c, SH_128x128, "eig/dc Q^T X", A2, X2, S2, n2, naux, n2, 1)));
  }
  hipLaunchKernelGGL(k_dc_prep, dim3(blocks_for(n)), dim3(256), 0, c->stream, d, n1, n2, E1, E2,
                     scal, ds, zs, src);
  CHECK(launch_check(c, "k_dc_prep"));
  hipLaunchKernelGGL(k_dc_gather_rows, dim3(blocks_for(naux), (unsigned)n), dim3(256), 0,
                     c->stream, G, src, n, naux, Gs);
  CHECK(launch_check(c, "k_dc_gather_rows"));
  hipLaunchKernelGGL(k_dc_deflate, dim3(1), dim3(256), 0, c->stream, ds, zs, n, scal, nd, dk, zk,
                     df, dfv, ra, rb, rc, rs, cnt);
  CHECK(launch_check(c, "k_dc_deflate"));
  int64_t hc[3] = {0, 0, 0};
  int hinfo[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(hinfo, flags + 1, sizeof(hinfo), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (hinfo[0] != 0 || hinfo[1] != 0)
    return fail(c, QSGW_ERR_SOLVER, "%s: dstedc info = %d, %d", what, hinfo[0], hinfo[1]);
  const int64_t K = hc[0], ndf = hc[1], nrot = hc[2];
  if (K < 0 || ndf < 0 || K + ndf != n || nrot < 0 || nrot > ndf)
    return fail(c, QSGW_ERR_SOLVER, "%s: deflation counts K = %lld, deflated = %lld", what,
                (long long)K, (long long)ndf);
  if (nrot > 0) {
    hipLaunchKernelGGL(k_dc_rotate, dim3(blocks_for(naux)), dim3(256), 0, c->stream, Gs, naux, ra,
                       rb, rc, rs, nrot);
    CHECK(launch_check(c, "k_dc_rotate"));
  }
  double* U = A;  // E1 and E2 are consumed
  if (K > 0) {
    hipLaunchKernelGGL(k_dc_secular, dim3(blocks_for(K, 4)), dim3(256), 0, c->stream, dk, zk, K,
                       scal, dor, mu, lam);
    CHECK(launch_check(c, "k_dc_secular"));
    hipLaunchKernelGGL(k_dc_zhat, dim3(blocks_for(K, 4)), dim3(256), 0, c->stream, dk, zk, K, scal,
                       dor, mu, zh);
    CHECK(launch_check(c, "k_dc_zhat"));
    hipLaunchKernelGGL(k_dc_vectors, dim3((unsigned)K), dim3(256), 0, c->stream, dk, zh, K, dor,
                       mu, U);
    CHECK(launch_check(c, "k_dc_vectors"));
  }
  if (ndf > 0) {
    hipLaunchKernelGGL(k_dc_sort_deflated, dim3(blocks_for(ndf)), dim3(256), 0, c->stream, dfv, df,
                       ndf, dfs, dfrow);
    CHECK(launch_check(c, "k_dc_sort_deflated"));
  }
  hipLaunchKernelGGL(k_dc_positions, dim3(blocks_for(n)), dim3(256), 0, c->stream, lam, K, dfs,
                     ndf, evals, posnd, posdf);
  CHECK(launch_check(c, "k_dc_positions"));
  double* Gnd = G;  // G is consumed (Gs holds its sorted rows)
  hipLaunchKernelGGL(k_dc_split_rows, dim3(blocks_for(naux), (unsigned)n), dim3(256), 0, c->stream,
                     Gs, nd, K, dfrow, posdf, ndf, naux, n, Gnd, R);
  CHECK(launch_check(c, "k_dc_split_rows"));
  if (K > 0) {
    // R[P][posnd[j]] = sum_i Gnd[i][P] U[j][i]
    Strided<false> Ag{Gnd, 1, naux, 0, naux};
    Strided<true> Bu{U, K, 1, 0, K};
    EpiScatterCols E{R, n, posnd};
    CHECK((gemm_shape<double, false>(c, SH_128x128, "eig/dc merge", Ag, Bu, E, naux, K, K, 1)));
  }
  return QSGW_OK;
}
