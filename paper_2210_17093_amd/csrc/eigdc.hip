// Tridiagonal stage of the two-stage Casida eigensolver in projection mode:
// divide and conquer whose merges are done here, on the projected columns
// only; the leaves (order <= the tile table's dc_leaf) are solved by rocSOLVER
// dstedc.
//
// A tridiagonal T (order n, diagonal d, off-diagonal e) is torn at
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
// n x q matrix), so E is never formed: R = U^T (Q^T X) with the rows of
// Q^T X sorted, rotated and split into deflated rows (copied to their
// columns of R) and the K others (one product with U).  Q^T X comes from the
// two halves solved the same way, each on its rows of X plus one unit column
// (e_{n1-1} for the first half, e_0 for the second): their projections are
// the boundary rows of E1 and E2 that z is made of.  Everything in FP64.
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

// The halves' eigenvalues (w = w1 of n1 then w2 of n2, each ascending)
// merged into ds ascending (ties: the first half first), with z unnormalised
// (the last row of E1 and sign(beta) times the first row of E2: row q of the
// halves' projections Rl [q + 1][n1] and Rr [q + 1][n2]) and the source row.
__global__ void k_dc_prep(const double* __restrict__ w, int64_t n1, int64_t n2,
                          const double* __restrict__ Rl, const double* __restrict__ Rr, int64_t q,
                          const double* __restrict__ scal, double* __restrict__ ds,
                          double* __restrict__ zs, int64_t* __restrict__ src) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n1 + n2) return;
  const double sg = scal[0] < 0.0 ? -1.0 : 1.0;
  int64_t pos;
  double v, z;
  if (t < n1) {
    v = w[t];
    pos = t + count_below(w + n1, n2, v, false);
    z = Rl[q * n1 + t];
  } else {
    const int64_t t2 = t - n1;
    v = w[n1 + t2];
    pos = t2 + count_below(w, n1, v, true);
    z = sg * Rr[q * n2 + t2];
  }
  ds[pos] = v;
  zs[pos] = z;
  src[pos] = t;
}

// Gs[s][P] = column src[s] of the halves' projections (Rl [.][n1] for
// src < n1, Rr [.][n2] after), P < q: a transpose through LDS in 64 x 64 tiles
// (reads along s, writes along P).
__global__ __launch_bounds__(256) void k_dc_gather_rows(const double* __restrict__ Rl,
                                                        const double* __restrict__ Rr, int64_t n1,
                                                        int64_t n2,
                                                        const int64_t* __restrict__ src,
                                                        int64_t q, double* __restrict__ Gs) {
  __shared__ double tile[64][65];
  const int64_t n = n1 + n2;
  const int64_t s0 = (int64_t)blockIdx.x * 64, P0 = (int64_t)blockIdx.y * 64;
  const int tid = threadIdx.x;
  const int sl = tid & 63, pr = tid >> 6;
  const int64_t s = s0 + sl;
  const int64_t t = s < n ? src[s] : 0;
  for (int pl = pr; pl < 64; pl += 4) {
    const int64_t P = P0 + pl;
    double v = 0.0;
    if (s < n && P < q) v = t < n1 ? Rl[P * n1 + t] : Rr[P * n2 + (t - n1)];
    tile[pl][sl] = v;
  }
  __syncthreads();
  for (int r = pr; r < 64; r += 4) {
    const int64_t s2 = s0 + r, P = P0 + sl;
    if (s2 < n && P < q) Gs[s2 * q + P] = tile[sl][r];
  }
}

// Inputs of the two halves of a node (X row-major [q][ldx], rows of T along
// the row): Xl [q + 1][n1] = first n1 entries of each row, then e_{n1-1};
// Xr [q + 1][n2] = the other n2 entries, then e_0.
__global__ void k_dc_child_inputs(const double* __restrict__ X, int64_t ldx, int64_t q, int64_t n1,
                                  int64_t n2, double* __restrict__ Xl, double* __restrict__ Xr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = blockIdx.y;
  if (P > q || r >= n1 + n2) return;
  if (r < n1)
    Xl[P * n1 + r] = P < q ? X[P * ldx + r] : (r == n1 - 1 ? 1.0 : 0.0);
  else
    Xr[P * n2 + (r - n1)] = P < q ? X[P * ldx + r] : (r == n1 ? 1.0 : 0.0);
}

// Deflation, one workgroup.  rho = |beta| |z|^2 and tol go to scal[1],
// scal[2]; then thread 0 walks the poles in order (staged through LDS in
// chunks, z normalised on the way) and emits the non-deflated poles (nd, dk,
// zk), the deflated ones (df, dfv) and the rotations (ra, rb, rc, rs) in the
// order they are to be applied.  cnt = {K, deflated, rotations}.  The
// non-deflated poles come out strictly increasing, every gap above 16 eps
// max |d| (a smaller one passes the rotation test and deflates), which the
// secular brackets rely on.
constexpr int kDcChunk = 2048;
__global__ __launch_bounds__(256) void k_dc_deflate(const double* __restrict__ ds,
                                                    const double* __restrict__ zs, int64_t n,
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


// Buffers of one recursion depth (one node of that depth is active at a time):
// the children's inputs Xc and projections Rc ([q + 1][n] each), the sorted
// and the non-deflated rows of Q^T X (Gs, Gnd: [n][q]), the vectors V and the
// int64 maps I of the merge.
struct DcLevel {
  double *Xc, *Rc, *Gs, *Gnd, *V;
  int64_t* I;
};
struct DcRun {
  std::vector<DcLevel> lv;
  int* info;  // one dstedc status per leaf
  int leaves = 0;
  int64_t leaf;  // leaves up to this order go to rocSOLVER dstedc
  const char* what;
};

// Merge of a node whose halves are solved: w (their eigenvalues, n1 then n2),
// Rl, Rr (their projections, [q + 1][n1], [q + 1][n2]), scal[0] = beta; out:
// evals (ascending) and R [q][n].  A: room for K x K.
static int dc_merge(qsgw_ctx* c, int64_t n1, int64_t n2, const double* w, const double* Rl,
                    const double* Rr, int64_t q, double* scal, const DcLevel& L, double* A,
                    double* evals, double* R, const char* what) {
  const int64_t n = n1 + n2;
  double* V = L.V;
  double *ds = V, *zs = V + n, *dk = V + 2 * n, *zk = V + 3 * n, *dfv = V + 4 * n, *rc = V + 5 * n,
         *rs = V + 6 * n, *dor = V + 7 * n, *mu = V + 8 * n, *lam = V + 9 * n, *zh = V + 10 * n,
         *dfs = V + 11 * n;
  int64_t* I = L.I;
  int64_t *src = I, *nd = I + n, *df = I + 2 * n, *ra = I + 3 * n, *rb = I + 4 * n,
          *dfrow = I + 5 * n, *posnd = I + 6 * n, *posdf = I + 7 * n, *cnt = I + 9 * n;
  double *Gs = L.Gs, *Gnd = L.Gnd;
  hipLaunchKernelGGL(k_dc_prep, dim3(blocks_for(n)), dim3(256), 0, c->stream, w, n1, n2, Rl, Rr, q,
                     scal, ds, zs, src);
  CHECK(launch_check(c, "k_dc_prep"));
  hipLaunchKernelGGL(k_dc_gather_rows, dim3(blocks_for(n, 64), blocks_for(q, 64)), dim3(256), 0,
                     c->stream, Rl, Rr, n1, n2, src, q, Gs);
  CHECK(launch_check(c, "k_dc_gather_rows"));
  hipLaunchKernelGGL(k_dc_deflate, dim3(1), dim3(256), 0, c->stream, ds, zs, n, scal, nd, dk, zk,
                     df, dfv, ra, rb, rc, rs, cnt);
  CHECK(launch_check(c, "k_dc_deflate"));
  int64_t hc[3] = {0, 0, 0};
  HIP_TRY(c, hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t K = hc[0], ndf = hc[1], nrot = hc[2];
  if (K < 0 || ndf < 0 || K + ndf != n || nrot < 0 || nrot > ndf)
    return fail(c, QSGW_ERR_SOLVER, "%s: deflation counts K = %lld, deflated = %lld", what,
                (long long)K, (long long)ndf);
  if (nrot > 0) {
    hipLaunchKernelGGL(k_dc_rotate, dim3(blocks_for(q)), dim3(256), 0, c->stream, Gs, q, ra, rb, rc,
                       rs, nrot);
    CHECK(launch_check(c, "k_dc_rotate"));
  }
  double* U = A;
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
  hipLaunchKernelGGL(k_dc_split_rows, dim3(blocks_for(q), (unsigned)n), dim3(256), 0, c->stream,
                     Gs, nd, K, dfrow, posdf, ndf, q, n, Gnd, R);
  CHECK(launch_check(c, "k_dc_split_rows"));
  if (K > 0) {
    // R[P][posnd[j]] = sum_i Gnd[i][P] U[j][i]
    Strided<false> Ag{Gnd, 1, q, 0, q};
    Strided<true> Bu{U, K, 1, 0, K};
    EpiScatterCols E{R, n, posnd};
    CHECK((gemm_shape<double, false>(c, SH_128x128, "eig/dc merge", Ag, Bu, E, q, K, K, 1)));
  }
  return QSGW_OK;
}

// Node of order n at recursion depth `depth`: T from d, e (destroyed), X row-major
// [q][ldx]; out: evals (ascending), R [q][n] with R[P][s] = sum_r E[r][s] X[P][r].
static int dc_node(qsgw_ctx* c, DcRun& run, int depth, int64_t n, double* d, double* e, double* A,
                   const double* X, int64_t ldx, int64_t q, double* evals, double* R) {
  if (n <= run.leaf) {
    rocblas_status st = rocsolver_dstedc(c->blas, rocblas_evect_tridiagonal, (rocblas_int)n, d, e,
                                         A, (rocblas_int)n, (rocblas_int*)(run.info + run.leaves));
    ++run.leaves;
    if (st != rocblas_status_success)
      return fail(c, QSGW_ERR_SOLVER, "%s: rocsolver_dstedc status %d", run.what, (int)st);
    // R[P][s] = sum_r X[P][r] E[r][s] (E column-major in A)
    Strided<true> Ax{X, ldx, 1, 0, q};
    Strided<true> Be{A, n, 1, 0, n};
    EpiStore S{R, n, 0, 0, 1.0};
    CHECK((gemm_shape<double, false>(c, SH_128x128, "eig/dc leaf", Ax, Be, S, q, n, n, 1)));
    HIP_TRY(c, hipMemcpyAsync(evals, d, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    return QSGW_OK;
  }
  const DcLevel& L = run.lv[(size_t)depth];
  const int64_t n1 = n / 2, n2 = n - n1;
  double* scal = L.V + 13 * n;
  double* w = L.V + 12 * n;  // the halves' eigenvalues
  hipLaunchKernelGGL(k_dc_tear, dim3(1), dim3(64), 0, c->stream, d, e, n1, scal);
  CHECK(launch_check(c, "k_dc_tear"));
  double *Xl = L.Xc, *Xr = L.Xc + (q + 1) * n1;
  double *Rl = L.Rc, *Rr = L.Rc + (q + 1) * n1;
  hipLaunchKernelGGL(k_dc_child_inputs, dim3(blocks_for(n), (unsigned)(q + 1)), dim3(256), 0,
                     c->stream, X, ldx, q, n1, n2, Xl, Xr);
  CHECK(launch_check(c, "k_dc_child_inputs"));
  CHECK(dc_node(c, run, depth + 1, n1, d, e, A, Xl, n1, q + 1, w, Rl));
  CHECK(dc_node(c, run, depth + 1, n2, d + n1, e + n1, A, Xr, n2, q + 1, w + n1, Rr));
  return dc_merge(c, n1, n2, w, Rl, Rr, q, scal, L, A, evals, R, run.what);
}

}  // namespace

// Eigenvalues (ascending) of the tridiagonal T (d, e: destroyed) and
// R[P][s] = sum_r E[r][s] X[P][r] for X row-major [naux][n] (column-major
// n x naux, ld n), without forming E.  A: n x n work array.
int tridiag_project_dc(qsgw_ctx* c, int64_t n, double* d, double* e, double* A, int64_t naux,
                       const double* X, double* evals, double* R, const char* what) {
  if (n < 4) return fail(c, QSGW_ERR_INVALID_ARG, "%s: tridiagonal merge needs n >= 4", what);
  // depth of the recursion (orders at depth l are at most ceil(n / 2^l))
  const int64_t leaf = c->tiles.dc_leaf;
  std::vector<int64_t> nl(1, n);
  while (nl.back() > leaf) nl.push_back(nl.back() - nl.back() / 2);
  const int depths = (int)nl.size() - 1;  // levels with a merge
  if (depths == 0) {
    // one leaf: still through the merge's interface (tear once)
    nl.push_back(n - n / 2);
  }
  const int nmerge = depths > 0 ? depths : 1;
  size_t big = 0, vec = 0, ints = 0;
  for (int l = 0; l < nmerge; ++l) {
    const size_t m = (size_t)nl[(size_t)l], q = (size_t)(naux + l);
    big += 2 * (q + 1) * m + 2 * m * q;
    vec += 13 * m + 8;
    ints += 9 * m + 4;
  }
  const int max_leaves = 1 << (nmerge + 1);
  double *B, *Vv;
  int64_t* Iv;
  CHECK(ws_get(c, W_EIG_DCG, big, &B));
  CHECK(ws_get(c, W_EIG_DCV, vec, &Vv));
  CHECK(ws_get(c, W_EIG_DCI, ints + (size_t)max_leaves, &Iv));
  DcRun run;
  run.what = what;
  run.leaf = leaf;
  for (int l = 0; l < nmerge; ++l) {
    const int64_t m = nl[(size_t)l], q = naux + l;
    DcLevel L;
    L.Xc = B;
    L.Rc = B + (q + 1) * m;
    L.Gs = B + 2 * (q + 1) * m;
    L.Gnd = L.Gs + m * q;
    B += 2 * (q + 1) * m + 2 * m * q;
    L.V = Vv;
    Vv += 13 * m + 8;
    L.I = Iv;
    Iv += 9 * m + 4;
    run.lv.push_back(L);
  }
  run.info = reinterpret_cast<int*>(Iv);
  HIP_TRY(c, hipMemsetAsync(run.info, 0, (size_t)max_leaves * sizeof(int64_t), c->stream));
  if (depths == 0) {
    // n <= dc_leaf: a single merge of two dstedc halves
    const DcLevel& L = run.lv[0];
    const int64_t n1 = n / 2, n2 = n - n1;
    double* scal = L.V + 13 * n;
    double* w = L.V + 12 * n;
    hipLaunchKernelGGL(k_dc_tear, dim3(1), dim3(64), 0, c->stream, d, e, n1, scal);
    CHECK(launch_check(c, "k_dc_tear"));
    double *Xl = L.Xc, *Xr = L.Xc + (naux + 1) * n1;
    double *Rl = L.Rc, *Rr = L.Rc + (naux + 1) * n1;
    hipLaunchKernelGGL(k_dc_child_inputs, dim3(blocks_for(n), (unsigned)(naux + 1)), dim3(256), 0,
                       c->stream, X, n, naux, n1, n2, Xl, Xr);
    CHECK(launch_check(c, "k_dc_child_inputs"));
    CHECK(dc_node(c, run, 1, n1, d, e, A, Xl, n1, naux + 1, w, Rl));
    CHECK(dc_node(c, run, 1, n2, d + n1, e + n1, A, Xr, n2, naux + 1, w + n1, Rr));
    CHECK(dc_merge(c, n1, n2, w, Rl, Rr, naux, scal, L, A, evals, R, what));
  } else {
    CHECK(dc_node(c, run, 0, n, d, e, A, X, n, naux, evals, R));
  }
  std::vector<int> hinfo((size_t)run.leaves, 0);
  HIP_TRY(c, hipMemcpyAsync(hinfo.data(), run.info, hinfo.size() * sizeof(int),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < run.leaves; ++i)
    if (hinfo[(size_t)i] != 0)
      return fail(c, QSGW_ERR_SOLVER, "%s: dstedc info = %d (leaf %d)", what, hinfo[(size_t)i], i);
  return QSGW_OK;
}
