// Element-wise, gather, reduction and pole-sum kernels of the qsGW iteration,
// plus the operand/epilogue functors that specialise the FP64 GEMM engine to
// each contraction.  All offsets are 64-bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.hpp"

namespace qsgw {

// ------------------------------------------------------------ operands ----
// Fock exchange in the MO basis, K_mn = sum_P sum_{i<nocc} B^P_{im} B^P_{in}:
// element (r = m, k = (P, i)) at B_mo[P][i][m]; m is unit-stride.
struct OccRowsOp {
  static constexpr bool kContig = false;
  const double* bmo;
  int64_t nbf, nocc;
  __device__ __forceinline__ double get(int64_t, int64_t r, int64_t k) const {
    if (r >= nbf) return 0.0;
    const int64_t P = k / nocc;
    const int64_t i = k - P * nocc;
    return bmo[(P * nbf + i) * nbf + r];
  }
};

// Pole-weighted residues for the qsGW matrix, Eqs. (17) and (19):
// element (r = m, k = (kst, s)) = w[m][kst][s] * Re 1/(eps_m - eps_kst +- (Omega_s - i eta))
//   = w * x / (x^2 + eta^2),  x = eps_m - eps_kst + Omega_s (occupied kst)
//                             x = eps_m - eps_kst - Omega_s (empty kst)
struct PoleScaledResidueOp {
  static constexpr bool kContig = true;
  const double* w;
  const double* eps;
  const double* Omega;
  int64_t nbf, nocc, ns;
  double eta;
  __device__ __forceinline__ double get(int64_t, int64_t r, int64_t k) const {
    if (r >= nbf) return 0.0;
    // k < nbf * ns < 2^32 (checked by the caller): 32-bit division
    const int64_t kst = (int64_t)((uint32_t)k / (uint32_t)ns);
    const int64_t s = k - kst * ns;
    const double om = Omega[s];
    const double x = eps[r] - eps[kst] + (kst < nocc ? om : -om);
    return w[r * nbf * ns + k] * (x / (x * x + eta * eta));
  }
};

// ----------------------------------------------------------- epilogues ----
// Casida matrix: M[t][u] = 4 v + delta_tu Delta_t^2, with v = sum_P Bt Bt
// where Bt = B_ia sqrt(Delta) already carries the (A-B)^{1/2} factors.
struct EpiCasida {
  double* Mout;
  const double* delta;
  int64_t ld;  // row pitch of Mout (ntr, or a padded order)
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t m, int64_t n, double v,
                                             bool mirror) const {
    double x = 4.0 * v;
    if (m == n) x += delta[m] * delta[m];
    Mout[m * ld + n] = x;
    if (mirror) Mout[n * ld + m] = x;
  }
};

// rho'[P][s] = sqrt(2 / Omega_s) v: the (X+Y) normalisation Omega^{-1/2} and
// the singlet spin factor sqrt(2) of Eq. (18) applied once per column.
struct EpiRho {
  double* rho;
  const double* Omega;  // already offset to the block's first excitation
  int64_t ld;
  float* rho32 = nullptr;  // optional FP32 copy
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t m, int64_t n, double v,
                                             bool) const {
    const double r = v * sqrt(2.0 / Omega[n]);
    rho[m * ld + n] = r;
    if (rho32) rho32[m * ld + n] = (float)r;
  }
};

// Residues from the pair-blocked product (rows = pair tiles of PairRows<8, 16>):
// w[m][k][s] for m <= k, mirrored to (k, m), so w is exactly symmetric in
// (m, k).  With wh != nullptr also the pole-weighted copy used by the qsGW
// matrix, Eqs. (17) and (19):
//   wh[m][k][s] = w[m][k][s] Re 1/(eps_m - eps_k +- (Omega_s - i eta)) = w x / (x^2 + eta^2),
//   x = eps_m - eps_k + Omega_s (occupied k) or eps_m - eps_k - Omega_s (empty k);
// the mirrored entry (k, m) gets its own weight.
struct EpiPairResidue {
  double* w;              // nullptr: not written (the FP32 variant keeps w32 only)
  double* wh;             // nullptr: residues only
  const int32_t* blocks;
  const double* eps;
  const double* Omega;    // the block's excitations
  int64_t nbf, nocc, ns;
  double eta;
  // FP32 variant of the qsGW product (both null otherwise): wh32 = the
  // pole-weighted copy with every near-pole term (|x| < thr) set to zero,
  // w32 = w rounded to FP32.  The near-pole terms are summed in FP64 apart.
  float* wh32 = nullptr;
  float* w32 = nullptr;
  double thr = 0.0;
  __device__ __forceinline__ double xval(int64_t a, int64_t b, double om) const {
    return eps[a] - eps[b] + (b < nocc ? om : -om);
  }
  // (the residues are written once and read by later kernels: non-temporal
  // stores keep them from evicting the product's operand panels from L2)
  __device__ __forceinline__ void store(int64_t a, int64_t b, int64_t s, double v) const {
    const int64_t i = (a * nbf + b) * ns + s;
    if (w) __builtin_nontemporal_store(v, &w[i]);
    if (wh) {
      const double x = xval(a, b, Omega[s]);
      __builtin_nontemporal_store(v * (x / (x * x + eta * eta)), &wh[i]);
    }
  }
  // Reduced-precision variants: the FP32 copies, with the pole weight of the
  // far terms in FP32 (x is formed in FP64, so the weight carries only the
  // FP32 rounding that its product is rounded to anyway).
  __device__ __forceinline__ void store32(int64_t a, int64_t b, int64_t s, double v, double om,
                                          float eta2) const {
    const int64_t i = (a * nbf + b) * ns + s;
    const double x = xval(a, b, om);
    const float xf = (float)x;
    const float vf = (float)v;
    const float g = xf * __builtin_amdgcn_rcpf(fmaf(xf, xf, eta2));
    if (w) __builtin_nontemporal_store(v, &w[i]);
    __builtin_nontemporal_store(fabs(x) >= thr ? vf * g : 0.0f, &wh32[i]);
    __builtin_nontemporal_store(vf, &w32[i]);
  }
  __device__ __forceinline__ void operator()(int64_t, int64_t, int64_t r, int64_t s, double v,
                                             bool) const {
    int64_t m, k;
    pair_of<8, 16>(blocks, r >> 7, (int)(r & 127), m, k);
    if (m >= nbf || k >= nbf || m > k) return;
    if (wh32) {
      const double om = Omega[s];
      const float eta2 = (float)(eta * eta);
      store32(m, k, s, v, om, eta2);
      if (m != k) store32(k, m, s, v, om, eta2);
      return;
    }
    store(m, k, s, v);
    if (m != k) store(k, m, s, v);
  }
};

// Split-BF16 variant of the residue epilogue.  For each pair (a, b) in
// {(m, k), (k, m)} and excitation s it writes
//   w[a][b][s] = w in FP64 if w is set,
//   wN[colidx[b][s]][a] = w in FP32 where colidx[b][s] >= 0 (the compacted
//                  near-pole columns the near-pole part reads),
// and the qsGW product's operands in the Split8 layout (rows a, k index
// j = b * nsp + s, nsp = ns rounded up to 8, s >= ns stored as zero):
//   ws  = w split into BF16 halves,
//   whs = w Re 1/(x -+ i eta) split the same way, zero where |x| < thr (those
//         terms are summed in FP64 apart), x = eps_a - eps_b +- Omega_s.
// It runs on the whole staged tile (kPassHook, FP32 staging): 128 pair rows
// (one pair block) by the tile's columns, eight excitations (one 16-byte
// chunk per plane) per work item, with the items ordered so that the chunks
// of consecutive threads are adjacent in memory (consecutive a).
struct EpiPairResidueX3 {
  static constexpr bool kPassHook = true;
  double* w;  // nullptr: not written
  float* wN;
  const int32_t* colidx;  // [nbf][nsp]
  uint16_t* ws;
  uint16_t* whs;
  int64_t cs, ps, nsp;  // Split8 rows per k-block slab, plane stride, padded ns
  const int32_t* blocks;
  const double* eps;
  const double* Omega;  // the block's excitations
  int64_t nbf, nocc, ns;
  double eta, thr;
  // (HAS_W: the FP64 residues are written too; without them no store of this
  // epilogue has the type of its FP64 loads, so loads of the next chunk can
  // move ahead of the stores of this one)
  template <bool HAS_W>
  __device__ __forceinline__ void put(int64_t a, int64_t b, int64_t s0, const double* v) const {
    const double ea = eps[a] - eps[b];
    const double sg = b < nocc ? 1.0 : -1.0;
    const float eta2 = (float)(eta * eta);
    const int4 ci0 = *reinterpret_cast<const int4*>(colidx + b * nsp + s0);
    const int4 ci1 = *reinterpret_cast<const int4*>(colidx + b * nsp + s0 + 4);
    const int ci[8] = {ci0.x, ci0.y, ci0.z, ci0.w, ci1.x, ci1.y, ci1.z, ci1.w};
    // (s0 is the same across each wave's work items: loaded as scalars)
    double om[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) om[u] = s0 + u < ns ? Omega[s0 + u] : 0.0;
    float wv[8], hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool ok = s0 + u < ns;
      const double x = ok ? ea + sg * om[u] : 1.0;
      const float xf = (float)x;
      const float vf = ok ? (float)v[u] : 0.0f;
      const float g = xf * __builtin_amdgcn_rcpf(fmaf(xf, xf, eta2));
      wv[u] = vf;
      hv[u] = fabs(x) >= thr ? vf * g : 0.0f;
    }
    // near-pole columns are rare: one wave-wide test skips the eight
    // conditional stores when no lane has any (columns past ns are never near)
    // (the AND keeps the sign bit only if every index is -1)
    const bool near = (ci[0] & ci[1] & ci[2] & ci[3] & ci[4] & ci[5] & ci[6] & ci[7]) >= 0;
    if (__any(near)) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (ci[u] >= 0) wN[(int64_t)ci[u] * nbf + a] = wv[u];
    }
    if (HAS_W) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (s0 + u < ns) w[(a * nbf + b) * ns + s0 + u] = v[u];
    }
    // The split operands (7.5 GB at N_b = 300) are written once and read by a
    // later kernel: non-temporal stores keep them from evicting the product's
    // own operand panels from L2.
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const int64_t o = ((b * nsp + s0) / 8 * cs + a) * 8;
    uint32_t h[4], l[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) split_bf16x2(wv[2 * u], wv[2 * u + 1], h[u], l[u]);
    __builtin_nontemporal_store(u32x4{h[0], h[1], h[2], h[3]}, reinterpret_cast<u32x4*>(ws + o));
    __builtin_nontemporal_store(u32x4{l[0], l[1], l[2], l[3]}, reinterpret_cast<u32x4*>(ws + ps + o));
#pragma unroll
    for (int u = 0; u < 4; ++u) split_bf16x2(hv[2 * u], hv[2 * u + 1], h[u], l[u]);
    __builtin_nontemporal_store(u32x4{h[0], h[1], h[2], h[3]}, reinterpret_cast<u32x4*>(whs + o));
    __builtin_nontemporal_store(u32x4{l[0], l[1], l[2], l[3]}, reinterpret_cast<u32x4*>(whs + ps + o));
  }
  // the whole tile: pair rows r0 .. r0 + 127 (one pair block: 8 values of m x
  // 16 of k), columns n0 .. n0 + BN - 1 at Cs[row * ldc + col]
  template <int ROWS, int BN>
  __device__ __forceinline__ void pass(int64_t r0, int64_t n0, const float* Cs, int ldc,
                                       int tid) const {
    if (w)
      pass_t<ROWS, BN, true>(r0, n0, Cs, ldc, tid);
    else
      pass_t<ROWS, BN, false>(r0, n0, Cs, ldc, tid);
  }
  template <int ROWS, int BN, bool HAS_W>
  __device__ __forceinline__ void pass_t(int64_t r0, int64_t n0, const float* Cs, int ldc,
                                         int tid) const {
    static_assert(ROWS == 128 && BN % 8 == 0, "one pair block of 8 x 16 pairs per tile");
    const int32_t bk = blocks[r0 >> 7];
    const int64_t mbase = (int64_t)(bk >> 16) * 8, kbase = (int64_t)(bk & 0xffff) * 16;
    constexpr int NSC = BN / 8, ITEMS = 128 * NSC;
    // (m, k): the eight m of one (k, chunk) fill one 128-byte line
    for (int q = tid; q < ITEMS; q += 256) {
      const int mo = q & 7, ko = (q >> 3) & 15;
      const int sc = __builtin_amdgcn_readfirstlane(q >> 7);  // one chunk per wave
      const int64_t m = mbase + mo, k = kbase + ko, s0 = n0 + 8 * sc;
      if (m >= nbf || k >= nbf || m > k || s0 >= ns) continue;
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = Cs[(mo * 16 + ko) * ldc + 8 * sc + u];
      put<HAS_W>(m, k, s0, v);
    }
    // (k, m), m < k: the sixteen k of one (m, chunk) fill two lines
    for (int q = tid; q < ITEMS; q += 256) {
      const int ko = q & 15, mo = (q >> 4) & 7;
      const int sc = __builtin_amdgcn_readfirstlane(q >> 7);  // one chunk per wave
      const int64_t m = mbase + mo, k = kbase + ko, s0 = n0 + 8 * sc;
      if (m >= nbf || k >= nbf || m >= k || s0 >= ns) continue;
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = Cs[(mo * 16 + ko) * ldc + 8 * sc + u];
      put<HAS_W>(k, m, s0, v);
    }
  }
};

// Near-pole terms of the qsGW product for one 64-row tile of m, over a
// compacted list of (k, s) columns (ktab, stab) that holds every pair with
// some m of the tile within thr of a pole:
//   A(r, j) = w[m][k][s] x / (x^2 + eta^2) if |x| < thr else 0,  m = m0 + r,
//   B(n, j) = w[n][k][s],   (k, s) = (ktab[j], stab[j]).
struct NearRowsOp {
  static constexpr bool kContig = true;
  const float* w;  // the FP32 copy of the residues (their accuracy is FP32 already)
  const double* eps;
  const double* Omega;
  const int32_t* ktab;
  const int32_t* stab;
  int64_t m0, rows, nbf, nocc, ns;
  double eta, thr;
  __device__ __forceinline__ double get(int64_t, int64_t r, int64_t j) const {
    if (r >= rows) return 0.0;
    const int64_t m = m0 + r, k = ktab[j], s = stab[j];
    const double x = eps[m] - eps[k] + (k < nocc ? Omega[s] : -Omega[s]);
    if (!(fabs(x) < thr)) return 0.0;
    return (double)w[(m * nbf + k) * ns + s] * (x / (x * x + eta * eta));
  }
};
struct NearColsOp {
  static constexpr bool kContig = true;
  const float* w;
  const int32_t* ktab;
  const int32_t* stab;
  int64_t nbf, ns;
  __device__ __forceinline__ double get(int64_t, int64_t n, int64_t j) const {
    if (n >= nbf) return 0.0;
    return (double)w[(n * nbf + ktab[j]) * ns + stab[j]];
  }
};

// ------------------------------------------------------ plain kernels ----

// Delta_t = eps_a - eps_i, sqrt_delta_t, and Bt[P][t] = B_mo[P][i][a] sqrt(Delta_t).
// ------------------------------------------------ per-state diagonal -----
// This thread's share of Eq. (17) with m = n at omega = eps_m, and of its
// frequency derivative, from row m of the residues (w[m][k][s], ns columns):
//   r[0] += sum w^2 x / (x^2 + eta^2)                      Re Sigma_mm(eps_m)
//   r[1] += sum (+-eta) w^2 / (x^2 + eta^2)                Im Sigma_mm(eps_m)
//   r[2] += -sum w^2 (x^2 - eta^2) / (x^2 + eta^2)^2       Re dSigma_mm/domega
// with x = eps_m - eps_k + Omega_s, +eta (occupied k) or x = eps_m - eps_k -
// Omega_s, -eta (empty k).  k runs outer, s is strided by the block size, so
// a wave reads consecutive addresses.
__device__ __forceinline__ void diag_self_partial(const double* wrow, const double* eps,
                                                  const double* Omega, int64_t m, int64_t nbf,
                                                  int64_t nocc, int64_t ns, double eta,
                                                  double r[3]) {
  const double em = eps[m], eta2 = eta * eta;
  for (int64_t k = 0; k < nbf; ++k) {
    const bool occ = k < nocc;
    const double base = em - eps[k];
    const double* wk = wrow + k * ns;
    for (int64_t s = threadIdx.x; s < ns; s += blockDim.x) {
      const double x = occ ? base + Omega[s] : base - Omega[s];
      const double w2 = wk[s] * wk[s];
      const double den = x * x + eta2;
      const double inv = 1.0 / den;
      r[0] += w2 * x * inv;
      r[1] += (occ ? eta : -eta) * w2 * inv;
      r[2] -= w2 * (x * x - eta2) * inv * inv;
    }
  }
}

// Sum of N values over the block (blockDim.x a multiple of 64, <= 1024), in a
// fixed order (wave shuffles, then waves in index order); valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(double v[N]) {
  __shared__ double red[16][N];
#pragma unroll
  for (int q = 0; q < N; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < N; ++q) red[threadIdx.x >> 6][q] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < N; ++q) {
      double t = 0.0;
      for (int u = 0; u < (int)(blockDim.x >> 6); ++u) t += red[u][q];
      v[q] = t;
    }
}

// One workgroup per listed state: out[j * ld + 0..2] (+)= the three sums of
// diag_self_partial for m = states[j] (m = j when states is null).
__global__ void k_sigma_diag_self(const double* w, const double* eps, const double* Omega,
                                  int64_t nbf, int64_t nocc, int64_t ns, double eta,
                                  const int64_t* states, int64_t nstates, double* out, int64_t ld,
                                  int accumulate, int* bad);

// Exchange diagonal in the MO basis, one workgroup per state m:
// out[m * ld] = -sum_{P, i < nocc} (B^P_mi)^2.
__global__ void k_exchange_diag(const double* bmo, int64_t naux, int64_t nbf, int64_t nocc,
                                double* out, int64_t ld);

// Exchange diagonal share of this thread for state m (P, i strided by the block).
__device__ __forceinline__ double exchange_diag_partial(const double* bmo, int64_t naux,
                                                        int64_t nbf, int64_t nocc, int64_t m) {
  double acc = 0.0;
  const int64_t n = naux * nocc;
  for (int64_t q = threadIdx.x; q < n; q += blockDim.x) {
    const int64_t P = q / nocc, i = q - P * nocc;
    const double b = bmo[(P * nbf + m) * nbf + i];
    acc -= b * b;
  }
  return acc;
}

// p[i] = v for i < n (a fill that graph capture records as a kernel node).
__global__ void k_fill(double* p, int64_t n, double v);

// Near-pole column ranges of the FP32 qsGW product.  For row tile t (rows
// [64 t, 64 t + 64) of m, energies ascending) and state k, the excitations s
// with |eps_m - eps_k +- Omega_s| < thr for some m of the tile form one
// contiguous range (Omega ascending): lo[t][k], cnt[t][k].  The range is
// widened by a relative 1e-12 so no near-pole term is missed; extra columns
// contribute zeros.
__global__ void k_near_ranges(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                              int64_t ns, double thr, int64_t ntiles, int64_t* lo, int64_t* cnt);

// Offsets of the (k, s) lists in order of k within each tile and each
// tile's total (one workgroup of at most 1024 threads per tile), then the
// tiles' starts base[t] in one table (k_near_bases, one thread, in order).
__global__ void k_near_offsets(const int64_t* cnt, int64_t nbf, int64_t ntiles, int64_t* off,
                               int64_t* total, int64_t* base);
__global__ void k_near_bases(const int64_t* total, int64_t ntiles, int64_t* base);

// Fill the compacted (k, s) lists: tile t's list starts at base[t].
__global__ void k_near_fill(const int64_t* lo, const int64_t* cnt, const int64_t* off,
                            const int64_t* base, int64_t nbf, int64_t ntiles, int32_t* ktab,
                            int32_t* stab);

__global__ void k_transitions(const double* eps, int64_t nocc, int64_t nv, double* delta,
                              double* sqrt_delta, int* bad);
// bt[P][t] = B_mo[P][i][a] sqrt_delta[t] for t = (i, a) (sqrt_delta NULL: unscaled)
__global__ void k_gather_bia(const double* bmo, const double* sqrt_delta, int64_t naux,
                             int64_t nbf, int64_t nocc, double* bt, float* bt32);
// Omega = sqrt(lambda); flags lambda <= 0 or non-finite.
__global__ void k_omega_from_eigs(const double* lam, int64_t n, double* Omega, int* bad);
// out[m][n] (+)= 1/2 (sum_z part[z][m][n] + sum_z part[z][n][m])
__global__ void k_reduce_sym(const double* part, int64_t nz, int64_t n, double* out, int accumulate);
// rho'[P][s] = sqrt(2 / Omega_s) sum_z part[z][P][s]  (split-K reduce of the rho product)
__global__ void k_rho_reduce(const double* part, int64_t nz, int64_t rows, int64_t ns,
                             const double* Omega, double* rho, float* rho32);

// out[i] = (float) in[i]
__global__ void k_to_f32(const double* in, int64_t n, float* out);

// Split-BF16 operands (Split8 layout, planes hi and lo, k-blocks of 8, K
// padded with zeros to kpad):
// rows of the residue product, one per pair (m, k) of the pair blocks
// (row t * 128 + i of block t), k = the auxiliary index P of B_mo[P][m][k];
// pairs outside the N x N range are zero.
__global__ void k_split_pairs(const double* bmo, const int32_t* blocks, int64_t nblk, int64_t nbf,
                              int64_t naux, int64_t kpad, uint16_t* out);
__global__ void k_zero_u16(uint16_t* p, int64_t n);

// Exact near-pole terms of the split-BF16 qsGW product (|x_mks| < thr with
// x_mks = (eps_m - eps_k) +- Omega_s, the residue epilogue's own formula).
// flag[k][s] (s < nsp) = 1 where some m has a near-pole term at (k, s).
__global__ void k_near_colflags(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                                int64_t ns, int64_t nsp, double thr, int64_t* flag);
// colidx[k][s] = base[k] + off[k][s] where flagged (the compacted column of
// (k, s), columns in (k, s) order), else -1.
__global__ void k_near_colidx(const int64_t* flag, const int64_t* off, const int64_t* base,
                              int64_t nbf, int64_t nsp, int32_t* colidx);
// For each (m, k): the near-pole excitations of (m, k) are s = slo .. slo + len - 1
// (contiguous, Omega ascending), their compacted columns c0 .. c0 + len - 1.
__global__ void k_near_mk(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                          int64_t ns, int64_t nsp, double thr, const int32_t* colidx,
                          int32_t* c0, int32_t* slo, int32_t* len);
// npart[z][m][n] = sum over k in [z kc, (z + 1) kc) and the near-pole s of
// (m, k) of w_mks Re 1/(x -+ i eta) w_nks, with w_nks = wN[column][n] (FP32
// columns the residue epilogue writes).  Grid (nbf, ceil(nbf / kc)),
// 256 threads, kc <= 64, nbf <= 2048.
__global__ void k_near_product(const double* eps, const double* Omega, int64_t nbf, int64_t nocc,
                               double eta, const int32_t* c0, const int32_t* slo,
                               const int32_t* len, const float* wN, int64_t kc, double* npart);
// out[g][e] = sum over slices z in [g zg, (g + 1) zg) of part[z][e] (e < len),
// g < ceil(nz / zg): the first, coalesced level of a long slice reduction.
__global__ void k_sum_slices(const double* part, int64_t nz, int64_t len, int64_t zg,
                             double* out);
// rows r < rows_pad of a [rows][ld] matrix read as (r, k) = in[r * ld + k]
// (r < rows, k < K; zero elsewhere).  Grid (rows_pad / 32, ceil(kpad / 256)),
// 256 threads; rows_pad a multiple of 32.
__global__ void k_split_rows(const double* in, int64_t ld, int64_t rows, int64_t K,
                             int64_t rows_pad, int64_t kpad, uint16_t* out);
// rows r < rows_pad of a [K][ld] matrix read as (r, k) = in[k * ld + r]
// (r < rows, k < K; zero elsewhere).
__global__ void k_split_cols(const double* in, int64_t ld, int64_t rows, int64_t K,
                             int64_t rows_pad, int64_t kpad, uint16_t* out);
// c_P = sum_{i<nocc} B_mo[P][i][i]
__global__ void k_occ_trace(const double* bmo, int64_t naux, int64_t nbf, int64_t nocc, double* c);
// J_mn = 2 sum_P c_P B_mo[P][m][n] in two levels: out[g][e] = 2 sum over
// P in [g pg, (g + 1) pg) of c_P bmo[P][e], then k_sum_slices over g.
__global__ void k_hartree_part(const double* bmo, const double* c, int64_t naux, int64_t nn,
                               int64_t pg, double* out);
// F[m][n] = sym(hmo)[m][n] + J[m][n] - sum_z Kpart[z][m][n] + V[m][n]
__global__ void k_fock_assemble(const double* hmo, const double* J, const double* Kpart, int64_t nz,
                                const double* V, int64_t n, double* F);
// X = diag(eps) - J + sum_z Kpart   (HF core in the MO basis)
__global__ void k_hf_core_mo(const double* eps, const double* J, const double* Kpart, int64_t nz,
                             int64_t n, double* X);
// out = 1/2 (a + a^T)
__global__ void k_symmetrize(const double* a, int64_t n, double* out);
// out = alpha * a + beta * b (elementwise)
__global__ void k_axpby(const double* a, const double* b, double alpha, double beta, int64_t len,
                        double* out);
// Sign convention of eigenvector columns: the largest-|.| entry is positive.
// Sign convention of eigenvector columns; launch one 256-thread workgroup per column.
__global__ void k_fix_column_signs(double* C, int64_t n);
// max_m |a_m - b_m| (one workgroup), and a finiteness flag.
__global__ void k_max_abs_diff(const double* a, const double* b, int64_t n, double* out);
// Non-finite scan: flags any NaN/Inf in x[0..len).
__global__ void k_check_finite(const double* x, int64_t len, int* bad, int mask);
// rho[P][s] *= sqrt(2 / Omega[s]) over a row-major [naux][ntr] array (the
// factor of Eq. (18) with the normalisation (X+Y)^s = sqrt(Delta) Z^s / sqrt(Omega_s))
__global__ void k_scale_rho(double* rho, int64_t naux, int64_t ntr, const double* Omega);
__global__ void k_check_finite_f32(const float* x, int64_t len, int* bad, int mask);
__global__ void k_bits_fingerprint(const double* x, int64_t len, unsigned long long* out);
__global__ void k_fock_frozen(const double* hmo, const double* V, int64_t n, double* F);
// Diagonal pole sum Sigma_mm(omega_l), Eq. (17), complex128 interleaved.
__global__ void k_sigma_diag_grid(const double* w, const double* eps, const double* Omega,
                                  int64_t nbf, int64_t nocc, int64_t ns, double eta,
                                  const double* omega, int64_t nomega, const int64_t* states,
                                  int64_t nstates, double* out, int accumulate, int* bad);

// qsMP2 right operand of one block of transitions (i in [i0, i0 + ni)):
// occupied p (flat grid over n, p, i, a) and empty p (32 x 32 LDS tiles).
__global__ void k_mp2_rhs_occ(const double* D, const double* xo, int64_t xsn, int64_t xsi,
                              const double* eps, int64_t nbf, int64_t nocc, int64_t i0,
                              int64_t ni, double eta, double* R);
__global__ void k_mp2_rhs_vir(const double* D, const double* eps, int64_t nbf, int64_t nocc,
                              int64_t i0, int64_t ni, double eta, double* R);

// Pulay DIIS on the Fock matrix (qsgw_iterate's optional accelerator of the
// fixed point).  The commutator error F D - D F of a Fock matrix F_mo given in
// the MO basis of the orbitals whose occupied block defines D: element
// (m, n) is F[m][n] (occ(n) - occ(m)), nonzero only between occupied and
// empty states.
__global__ void k_diis_error_mo(const double* F, int64_t n, int64_t nocc, double* out);
// B[k][j] = B[j][k] = <E_k, E_j>_F for the stored slots j (one workgroup per
// slot j in `slots`, fixed-order reduction); E is [m][len], B is [ld][ld].
__global__ void k_diis_dots(const double* E, int64_t len, int64_t k, const int* slots, double* B,
                            int64_t ld);
// Pulay weights: c minimising || sum_j c_j E_j || subject to sum_j c_j = 1,
// from the bordered (nact + 1) system over the slots in `slots` (one thread,
// Gaussian elimination with partial pivoting); c[i] is slot slots[i]'s weight.
// A singular system sets *bad and leaves the weight of the newest slot 1.
__global__ void k_diis_solve(const double* B, int64_t ld, const int* slots, int nact, double* c,
                             int* bad);
// out[e] = sum_i c[i] F[slots[i]][e], i in fixed order.
__global__ void k_diis_combine(const double* F, int64_t len, const int* slots, int nact,
                               const double* c, double* out);

// Open shell: one spin's transitions into the concatenated [naux][ld] tensor.
__global__ void k_gather_bia_ld(const double* bmo, const double* sqrt_delta, double scale,
                                int64_t naux, int64_t nbf, int64_t nocc, int64_t ld, double* bt);

}  // namespace qsgw
