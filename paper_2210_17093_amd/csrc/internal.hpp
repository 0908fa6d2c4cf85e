// Host-side machinery shared by the single-problem and batched drivers of
// libqsgw: the context, its workspace, error handling, GEMM launchers and
// K-split plans, stage timers, the pair-block table of the residue product
// and the dense eigensolver wrapper.
#pragma once
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>
#include <string>
#include <vector>

#include "../../include/qsgw.h"
#include "gemm_f64.hpp"
#include "kernels.hpp"

using namespace qsgw;

namespace {

enum Slot {
  W_T = 0,    // AO->MO half transform B_ao C            [naux][nbf][nbf]
  W_BMO,      // MO tensor (iterate / hf_core)            [naux][nbf][nbf]
  W_BT,       // B_ia sqrt(Delta)                         [naux][ntr]
  W_DELTA,    // Delta_t                                  [ntr]
  W_SQD,      // sqrt(Delta_t)                            [ntr]
  W_M,        // Casida matrix, then eigenvectors         [ntr][ntr]
  W_OMEGA,    // Omega                                    [ntr]
  W_RHO,      // rho' of one excitation block             [naux][sb]
  W_W,        // residues of one excitation block         [nbf][nbf][sb]
  W_WH,       // pole-weighted residues of the block      [nbf][nbf][sb]
  W_PART,     // split-K partial sums                     [nz][nbf][nbf]
  W_V,        // qsGW potential, MO basis                 [nbf][nbf]
  W_HMO,      // C^T h C                                  [nbf][nbf]
  W_J,        // Hartree, MO basis                        [nbf][nbf]
  W_CP,       // occupied traces c_P                      [naux]
  W_F,        // Fock, then its eigenvectors              [nbf][nbf]
  W_TMP,      // scratch                                  [nbf][nbf]
  W_TMP2,     // scratch                                  [nbf][nbf]
  W_EPSN,     // new energies                             [nbf]
  W_CNEW,     // new coefficients                         [nbf][nbf]
  W_EIGE,     // dsyevd off-diagonal workspace            [max(ntr, nbf)]
  W_SCAL,     // device scalars                           [8]
  W_FLAGS,    // device int flags                         [8]
  W_DIIS_F,   // DIIS history: AO Fock matrices             [m][nbf][nbf]
  W_DIIS_E,   // DIIS history: their commutator errors       [m][nbf][nbf]
  W_DIIS_B,   // DIIS error dot products                     [16][16]
  W_DIIS_X,   // DIIS weights, then the combined Fock matrix [nbf][nbf]
  W_DIIS_S,   // DIIS slots in time order (int)              [16]
  W_ROWTAB,   // residue pair blocks holding some m <= k  [blocks]
  W_RHOPART,  // split-K partial sums of rho              [nz][naux][sb]
  W_BATCH_F64,   // batched iteration: every molecule's arrays
  W_BATCH_I32,   // batched iteration: pair tables, flags, solver info
  W_BATCH_PRE,   // batched iteration: segment prefix sums, split counts
  W_BATCH_JOBS,  // batched iteration: grouped GEMM job tables
  W_BATCH_MOLS,  // batched iteration: molecule descriptors
  W_MLP_F32,     // warm-start network: activations, gradients
  W_MLP_F64,     // warm-start network: partial sums, squared errors
  W_MLP_PERM,    // warm start: state permutation
  W_NEAR,        // reduced-precision qsGW product: near-pole ranges, offsets, flags (int64)
  W_NEARTAB,     // reduced-precision qsGW product: near-pole column tables (int32)
  W_BMO32,       // FP32 products: B_mo rounded to FP32           [naux][nbf][nbf] float
  W_RHO32,       // FP32 products: rho' rounded to FP32           [naux][sb] float
  W_BT32,        // FP32 products: Bt rounded to FP32             [naux][ntr] float
  W_Z32,         // FP32 products: eigenvectors of a block, FP32  [sb][ntr] float
  W_SPLIT_A,     // split-BF16 residue product: B_mo pair rows    [2][kpad/8][pair rows][8] bf16
  W_SPLIT_B,     // split-BF16 residue product: rho' of a block   [2][kpad/8][sb padded][8] bf16
  W_SPLIT_W,     // split-BF16 qsGW product: w and wh of a block  [2][2][kfar/8][nbf padded][8] bf16
  W_SPLIT_CAS,   // split-BF16 Casida build: Bt, rows t, k = P     [2][naux/8][ntr padded][8] bf16
  W_SPLIT_RA,    // split-BF16 rho' product: Bt, rows P, k = t     [2][ntr/8][naux padded][8] bf16
  W_SPLIT_Z,     // split-BF16 rho' product: Z of a block, rows s  [2][ntr/8][sb padded][8] bf16
  W_NEARW,       // split-BF16 qsGW product: near-pole columns    [columns][nbf] float
  W_REDPART,     // first level of a long split-K reduction       [ceil(nz / 32)][nbf][nbf]
  W_MP2_BIA,     // qsMP2: B_mo[P][i][a], unscaled                [naux][ntr]
  W_MP2_D,       // qsMP2: (mp|ia) of a block of transitions     [nbf][nbf][block]
  W_MP2_R,       // qsMP2: pole-weighted right operand            [nbf][nbf][block]
  W_MP2_E,       // qsMP2, several blocks: (ni|pa), i occupied    [nocc][nbf][ntr]
  W_AO2MO,       // four-index AO->MO: quarter-transformed slab   [m_count][nbf][nbf][nbf]
  W_M2,          // replayed iteration: Casida matrix, checked against the solved one [ntr][ntr]
  W_FPRINT,      // bit fingerprints of Casida matrices           [2] u64
  W_EIG_V1,      // two-stage eigensolver: panel reflectors V    [sum of panel rows * b]
  W_EIG_T1,      // two-stage eigensolver: panel factors T       [panels][b][b]
  W_EIG_TAU1,    // two-stage eigensolver: panel tau             [panels][b]
  W_EIG_U,       // two-stage eigensolver: [V W], [W V]          [2][n][2b]
  W_EIG_XY,      // two-stage eigensolver: X, Y, small products   [2 n b + 2 b b]
  W_EIG_BAND,    // two-stage eigensolver: lower band + bulge     [n][2b+1]
  W_EIG_V2,      // two-stage eigensolver: bulge reflectors       [steps][b]
  W_EIG_TAU2,    // two-stage eigensolver: bulge tau              [steps]
  W_EIG_OFF,     // two-stage eigensolver: first step of a sweep  [n] int64
  W_EIG_DE,      // two-stage eigensolver: tridiagonal d, e       [2 n]
  W_EIG_TB,      // two-stage eigensolver: WY factors of the bulge reflector blocks [blocks][64][64]
  W_EIG_PX,      // two-stage projection: Q2^T Q1^T Bt^T          [naux][ntr]
  W_EIG_XP,      // two-stage eigensolver: split-K partials of X = S V T [nz][b][m]
  W_EIG_PANEL,   // two-stage eigensolver: panel QR partial dots (two buffers) and R  [2 G b + b b]
  W_EIG_Q1W,     // two-stage eigensolver: V^T X and T V^T X of a panel [2][b][ncols]
  W_EIG_PFLAG,   // two-stage eigensolver: cooperative panel QR barrier flags [256] u64, error flag
  W_EIG_DCG,     // tridiagonal merge (projection): Q^T X and its sorted rows [2][n][naux]
  W_EIG_DCV,     // tridiagonal merge: poles, weights, roots, rotations [12 n + 8]
  W_EIG_DCI,     // tridiagonal merge: row maps, positions, counts (int64) [9 n + 4]
  W_RHOFULL,     // iteration through the projection: rho' of every excitation [naux][ntr]
  W_RHOFULL32,   // ... and its FP32 copy (FP32 products)          [naux][ntr] float
  W_BMO_B,       // open-shell iteration: beta-spin MO tensor     [naux][nbf][nbf]
  W_VB,          // open-shell iteration: beta-spin potential     [nbf][nbf]
  W_NSLOTS
};

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

// Tile shapes of the tunable products (qsgw_set_tiles).  Symmetric (upper
// tile) products take square shapes only.
enum Shape { SH_64x64 = 0, SH_128x64 = 1, SH_128x128 = 2, SH_COUNT };
enum Tunable { TU_MO1 = 0, TU_MO2, TU_CASIDA, TU_RHO, TU_SIGMA, TU_EXCHANGE, TU_COUNT };
struct Tiles {
  int shape[TU_COUNT] = {SH_128x64, SH_64x64, SH_128x128, SH_128x128, SH_64x64, SH_64x64};
  // workgroups a K-split aims for when the output tiles alone are few
  int64_t sigma_target = 4096, rho_target = 2048, exchange_target = 2048;
  // the qsMP2 contraction (K = nbf * block transitions) wants more splits
  int64_t mp2_target = 32768;
  // batched grouped products: 0 = one workgroup per tile, n > 0 = a
  // persistent grid of n workgroups per compute unit walking tile ranges
  int64_t persistent = 0;
  // projected divide and conquer of the two-stage eigensolver: tridiagonal
  // blocks up to this order are solved by rocSOLVER dstedc
  int64_t dc_leaf = 6144;
  // two-stage eigensolver: 1 = panel QR in one cooperative launch per panel
  // (the per-column launches when the device refuses it), 0 = per-column launches
  int64_t panel_coop = 1;
};
inline int shape_m(int s) { return s == SH_64x64 ? 64 : 128; }
inline int shape_n(int s) { return s == SH_128x128 ? 128 : 64; }

}  // namespace

struct qsgw_ctx {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  rocblas_handle blas = nullptr;
  std::string err;
  Buffer ws[W_NSLOTS];
  std::vector<hipEvent_t> events;
  double stage_ms[7] = {0, 0, 0, 0, 0, 0, 0};
  // events bracketing each stage of the last single-stage call
  int last_stage = -1;
  // cached residue pair-block table
  int64_t rowtab_nbf = -1, rowtab_n = 0;
  Tiles tiles;
  // auxiliary streams (default priority) with their own rocBLAS handles, so
  // the bucketed eigensolves of the batched iteration overlap; created on
  // first use
  static constexpr int kAux = 3;
  hipStream_t aux[kAux] = {};
  rocblas_handle aux_blas[kAux] = {};
  hipEvent_t fork = nullptr, join[kAux] = {};
  bool aux_ready = false;
  // The last Casida matrix qsgw_iterate solved: its size (-1: none kept) and
  // bit fingerprint; W_M then holds its eigenvectors and W_OMEGA its
  // excitation energies (QSGW_OPT_REPLAY_EIG reads them).
  int64_t eig_ntr = -1;
  unsigned long long eig_fp = 0;
  // the kept eigenpairs are (Omega, rho' of every excitation in W_RHOFULL)
  // from the two-stage projection instead of (Omega, Z in W_M)
  bool eig_fold = false;
  // solver of the Casida eigenproblems (QSGW_EIG_*)
  int eig_solver = QSGW_EIG_AUTO;
  // this device's copy of the allocation-free entry point's static scratch
  // array (noalloc.hip), null if the lookup failed
  double* scratch = nullptr;
  // DIIS history of qsgw_iterate (W_DIIS_*): stored pairs, next slot, and
  // the (N_b, subspace size) it belongs to; diis_slots stages the slot order
  int64_t diis_n = 0, diis_next = 0, diis_nbf = -1, diis_m = 0;
  int diis_slots[16] = {};
};

// Looks up the device address of the static scratch array of the
// allocation-free entry point for the context's device (noalloc.hip).
int noalloc_setup(qsgw_ctx* c);

// Two-stage dense symmetric eigensolver (eig2s.hip): A [n][n] in, its
// eigenvectors column-major out, eigenvalues ascending.
int eig_two_stage(qsgw_ctx* c, int64_t n, double* A, double* evals, const char* what);
// Eigenvalues of A and R[P][s] = sum_t Bt[P][t] Z[t][s] without forming Z
// (eig2s.hip); A is destroyed, X is an [naux][n] work array.
int eig_two_stage_project(qsgw_ctx* c, int64_t n, double* A, double* evals, int64_t naux,
                          const double* Bt, double* X, double* R, const char* what);
// Eigenvalues (ascending) of a tridiagonal matrix (d, e: destroyed) and
// R[P][s] = sum_r E[r][s] X[P][r] (E its eigenvectors, X row-major [naux][n])
// by one divide-and-conquer merge of the two halves (eigdc.hip); A: n x n work.
int tridiag_project_dc(qsgw_ctx* c, int64_t n, double* d, double* e, double* A, int64_t naux,
                       const double* X, double* evals, double* R, const char* what);

// qsMP2 potential of Eqs. (20)-(21) in the MO basis (mp2.hip), for the
// iteration driver: V (+)= the potential; occ_block 0 = automatic blocks.
int qsgw_mp2_stage(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                   const double* eps, double eta, double* V, int64_t occ_block, int accumulate);

namespace {

constexpr int kStageMo = 0, kStageRpa = 1, kStageEigRpa = 2, kStageRes = 3, kStageSigma = 4,
              kStageFock = 5, kStageEigFock = 6;

int fail(qsgw_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, QSGW_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                       \
  } while (0)

#define CHECK(x)                \
  do {                          \
    int r_ = (x);               \
    if (r_ < 0) return r_;      \
  } while (0)

template <class T>
int ws_get(qsgw_ctx* c, int slot, size_t count, T** out) {
  const size_t bytes = count * sizeof(T) > 0 ? count * sizeof(T) : 8;
  Buffer& b = c->ws[slot];
  if (b.bytes < bytes) {
    if (b.p) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      HIP_TRY(c, hipFree(b.p));
      b.p = nullptr;
      b.bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, QSGW_ERR_ALLOC, "workspace allocation of %zu bytes failed (slot %d)", bytes,
                  slot);
    }
    b.p = p;
    b.bytes = bytes;
  }
  *out = static_cast<T*>(b.p);
  return QSGW_OK;
}

inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

int launch_check(qsgw_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, QSGW_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return QSGW_OK;
}

// K-split plan: chunks of a multiple of 16, no empty split.
struct SplitPlan {
  int64_t kchunk, nz;
};
inline SplitPlan split_plan(int64_t K, int64_t want) {
  if (want <= 1 || K <= 16) return {K, 1};
  int64_t kchunk = (K + want - 1) / want;
  kchunk = ((kchunk + 15) / 16) * 16;
  return {kchunk, (K + kchunk - 1) / kchunk};
}

// Launch the FP64 GEMM engine.  TRI requires M == N.  `sp` is the K-split plan
// (partial-sum buffers must hold sp.nz slices).
template <class T, int BM, int BN, bool TRI, int BK = 16, class OA, class OB, class EPI,
          class FILT = AllTiles>
int gemm_t(qsgw_ctx* c, const char* what, OA a, OB b, EPI e, int64_t M, int64_t N, int64_t K,
           int64_t batch, SplitPlan sp = {0, 1}, FILT f = FILT()) {
  const int64_t tm = (M + BM - 1) / BM;
  const int64_t tn = (N + BN - 1) / BN;
  const int64_t ntiles = TRI ? tm * (tm + 1) / 2 : tm * tn;
  const int64_t kchunk = sp.nz > 1 ? sp.kchunk : K;
  const int64_t splits = sp.nz > 1 ? sp.nz : 1;
  if (ntiles <= 0 || batch <= 0 || K <= 0) return QSGW_OK;
  const int64_t total = ntiles * batch * splits;
  if (total > 0x7fffffffLL) return fail(c, QSGW_ERR_INVALID_ARG, "%s: launch grid too large", what);
  constexpr bool kb = is_bf16x3<T>::value;
  if (!loader_offsets_fit(a, BM, BK, kb) || !loader_offsets_fit(b, BN, BK, kb))
    return fail(c, QSGW_ERR_UNSUPPORTED, "%s: operand strides too large for the tile loader", what);
  if (sp.nz > 1 && sp.kchunk % BK != 0)
    return fail(c, QSGW_ERR_INVALID_ARG, "%s: K chunk not a multiple of the k tile", what);
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, OA, OB, EPI, TRI, FILT, BK, T>), dim3((unsigned)total),
                     dim3(256), 0, c->stream, a, b, e, M, N, K, kchunk, tm, tn, batch, f);
  return launch_check(c, what);
}

// FP64 products.
template <int BM, int BN, bool TRI, class OA, class OB, class EPI, class FILT = AllTiles>
int gemm(qsgw_ctx* c, const char* what, OA a, OB b, EPI e, int64_t M, int64_t N, int64_t K,
         int64_t batch, SplitPlan sp = {0, 1}, FILT f = FILT()) {
  return gemm_t<double, BM, BN, TRI>(c, what, a, b, e, M, N, K, batch, sp, f);
}

// Longest K run one FP32-accumulating workgroup covers before its partial
// sum is handed to the FP64 split-K reduction.
constexpr int64_t kFp32MaxK = 4096;

// Split count that gives roughly `target` workgroups for a tiny output.
inline int64_t splits_for(int64_t tiles, int64_t K, int64_t target = 2048) {
  int64_t s = (target + tiles - 1) / tiles;
  const int64_t maxs = (K + 255) / 256;  // keep >= 256 k per split
  if (s > maxs) s = maxs;
  return s < 1 ? 1 : s;
}

inline int64_t tiles_of(int shape, int64_t M, int64_t N) {
  return ((M + shape_m(shape) - 1) / shape_m(shape)) * ((N + shape_n(shape) - 1) / shape_n(shape));
}

// qsGW matrix: tiles of the nbf x nbf output, K = nbf * ns.
inline SplitPlan sigma_split(const Tiles& tl, int64_t nbf, int64_t ns) {
  const int64_t t = tiles_of(tl.shape[TU_SIGMA], nbf, nbf);
  return split_plan(nbf * ns, splits_for(t, nbf * ns, tl.sigma_target));
}

// FP32 qsGW product: far-from-pole part on FP32 matrix cores (each split's
// K <= kFp32MaxK), near-pole part in FP64 over compacted columns, one 64-row
// tile of m at a time, in `near` extra partial slices.
constexpr double kNearPoleDefault = 0.05;  // Ha
// (K = the product's k length: nbf * ns, or x3_kfar for split operands)
inline SplitPlan sigma_split32(const Tiles& tl, int64_t nbf, int64_t K) {
  const int64_t t = tiles_of(tl.shape[TU_SIGMA], nbf, nbf);
  int64_t want = splits_for(t, K, tl.sigma_target);
  const int64_t need = (K + kFp32MaxK - 1) / kFp32MaxK;
  if (want < need) want = need;
  return split_plan(K, want);
}
inline int64_t near_slices_max(int64_t nbf) {
  const int64_t t = (nbf + 63) / 64;
  const int64_t z = (2048 + t * t - 1) / (t * t);
  return z < 1 ? 1 : z;
}
// k length of the split-BF16 qsGW product: k index j = k * nsp + s with ns
// padded to nsp (a multiple of 8), then to a multiple of the k tile (32).
inline int64_t x3_kfar(int64_t nbf, int64_t ns) {
  const int64_t nsp = (ns + 7) / 8 * 8;
  return (nbf * nsp + 31) / 32 * 32;
}
// split-BF16 near-pole part: k in slices of kX3NearK, one partial slice each
constexpr int64_t kX3NearK = 32;
inline int64_t x3_near_slices(int64_t nbf) { return (nbf + kX3NearK - 1) / kX3NearK; }
inline int64_t sigma_slices(const Tiles& tl, int64_t nbf, int64_t ns, bool fp32, bool x3 = false) {
  if (!fp32) return sigma_split(tl, nbf, ns).nz;
  if (x3) return sigma_split32(tl, nbf, x3_kfar(nbf, ns)).nz + x3_near_slices(nbf);
  return sigma_split32(tl, nbf, nbf * ns).nz + near_slices_max(nbf);
}

// qsMP2 potential: occupied states per block of transitions (occ_block 0:
// the largest block whose two [nbf][nbf][block transitions] FP64 work arrays
// fit in 16 GiB) and the K-split of its contraction (K = nbf * block transitions).
inline int64_t mp2_block(int64_t nbf, int64_t nocc, int64_t occ_block) {
  constexpr double kMp2BlockBytes = 16.0 * 1024 * 1024 * 1024;
  int64_t ib = occ_block;
  if (ib <= 0) {
    ib = (int64_t)(kMp2BlockBytes / (2.0 * 8.0 * (double)(nbf * nbf) * (double)(nbf - nocc)));
    if (ib < 1) ib = 1;
  }
  return ib > nocc ? nocc : ib;
}
inline SplitPlan mp2_split(const Tiles& tl, int64_t nbf, int64_t ntb) {
  return split_plan(nbf * ntb, splits_for(tiles_of(tl.shape[TU_SIGMA], nbf, nbf), nbf * ntb,
                                          tl.mp2_target));
}

// rho product: tiles of the naux x ns output, K = ntr; split only when the
// tiles alone leave the chip under-filled.
inline SplitPlan rho_split(const Tiles& tl, int64_t naux, int64_t ns, int64_t ntr, int64_t maxk) {
  const int64_t tiles = tiles_of(tl.shape[TU_RHO], naux, ns);
  int64_t want = tiles >= tl.rho_target ? 1 : splits_for(tiles, ntr, tl.rho_target);
  const int64_t need = (ntr + maxk - 1) / maxk;  // keep each split's K <= maxk
  if (want < need) want = need;
  return split_plan(ntr, want);
}

// MO exchange: upper square tiles, K = naux * nocc.
inline SplitPlan exchange_split(const Tiles& tl, int64_t nbf, int64_t naux, int64_t nocc) {
  const int64_t t = (nbf + shape_m(tl.shape[TU_EXCHANGE]) - 1) / shape_m(tl.shape[TU_EXCHANGE]);
  return split_plan(naux * nocc, splits_for(t * (t + 1) / 2, naux * nocc, tl.exchange_target));
}

// GEMM with the tile shape chosen at run time (BK: k-tile depth).
template <class T, bool TRI, int BK = 16, class OA, class OB, class EPI>
int gemm_shape(qsgw_ctx* c, int shape, const char* what, OA a, OB b, EPI e, int64_t M, int64_t N,
               int64_t K, int64_t batch, SplitPlan sp = {0, 1}) {
  switch (shape) {
    case SH_64x64:
      return gemm_t<T, 64, 64, TRI, BK>(c, what, a, b, e, M, N, K, batch, sp);
    case SH_128x128:
      return gemm_t<T, 128, 128, TRI, BK>(c, what, a, b, e, M, N, K, batch, sp);
    default:
      if constexpr (TRI) {
        return fail(c, QSGW_ERR_INVALID_ARG, "%s: symmetric products take square tiles", what);
      } else {
        return gemm_t<T, 128, 64, false, BK>(c, what, a, b, e, M, N, K, batch, sp);
      }
  }
}

// A K-split plan with chunks rounded up to a multiple of `bk`.
inline SplitPlan round_chunks(SplitPlan sp, int64_t K, int64_t bk) {
  if (sp.nz <= 1) return sp;
  sp.kchunk = ((sp.kchunk + bk - 1) / bk) * bk;
  sp.nz = (K + sp.kchunk - 1) / sp.kchunk;
  return sp;
}

int record(qsgw_ctx* c, size_t idx) {
  while (c->events.size() <= idx) {
    hipEvent_t e;
    HIP_TRY(c, hipEventCreate(&e));
    c->events.push_back(e);
  }
  HIP_TRY(c, hipEventRecord(c->events[idx], c->stream));
  return QSGW_OK;
}

double elapsed(qsgw_ctx* c, size_t a, size_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, c->events[a], c->events[b]) != hipSuccess) {
    (void)hipGetLastError();
    return 0.0;
  }
  return (double)ms;
}

// Timed spans on the context stream: each span is a pair of events; `id`
// names a stage (0..6) or a kernel (kKernelBase + 0..7).
constexpr int kKernelBase = 100;
constexpr int kKMo1 = kKernelBase + 0, kKMo2 = kKernelBase + 1, kKCasida = kKernelBase + 2,
              kKRho = kKernelBase + 3, kKW = kKernelBase + 4, kKSigma = kKernelBase + 5,
              kKSigmaRed = kKernelBase + 6, kKFock = kKernelBase + 7;

struct Spans {
  qsgw_ctx* c = nullptr;
  size_t next = 0;
  struct Span {
    int id;
    size_t e0, e1;
  };
  std::vector<Span> v;
  std::vector<size_t> open_stack;
  int open(int id) {
    if (!c) return QSGW_OK;
    v.push_back({id, next, 0});
    open_stack.push_back(v.size() - 1);
    return record(c, next++);
  }
  int close() {
    if (!c) return QSGW_OK;
    v[open_stack.back()].e1 = next;
    open_stack.pop_back();
    return record(c, next++);
  }
};

#define SPAN_OPEN(sp, id)              \
  do {                                 \
    if (sp) CHECK((sp)->open(id));     \
  } while (0)
#define SPAN_CLOSE(sp)                 \
  do {                                 \
    if (sp) CHECK((sp)->close());      \
  } while (0)

// Pair blocks (8 values of m x 16 values of k) of the residue product that
// hold at least one pair m <= k, encoded mb << 16 | kb, in row-major block
// order.  Built on the host once per nbf and kept on the device.
int pair_blocks(qsgw_ctx* c, int64_t nbf, const int32_t** tab, int64_t* n) {
  if (c->rowtab_nbf != nbf) {
    const int64_t nmb = (nbf + 7) / 8, nkb = (nbf + 15) / 16;
    if (nmb > 0x7fff || nkb > 0xffff) return fail(c, QSGW_ERR_INVALID_ARG, "nbf too large");
    std::vector<int32_t> keep;
    for (int64_t mb = 0; mb < nmb; ++mb)
      for (int64_t kb = 0; kb < nkb; ++kb)
        if (8 * mb <= 16 * kb + 15) keep.push_back((int32_t)((mb << 16) | kb));
    int32_t* d = nullptr;
    CHECK(ws_get(c, W_ROWTAB, keep.size(), &d));
    // work already queued may still read the previous table
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(d, keep.data(), keep.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    c->rowtab_nbf = nbf;
    c->rowtab_n = (int64_t)keep.size();
  }
  *tab = static_cast<const int32_t*>(c->ws[W_ROWTAB].p);
  *n = c->rowtab_n;
  return QSGW_OK;
}

int read_flag(qsgw_ctx* c, int* dflag, int* out) {
  HIP_TRY(c, hipMemcpyAsync(out, dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return QSGW_OK;
}

// rocSOLVER dsyevd, eigenvectors in place (column-major).
int syevd(qsgw_ctx* c, int64_t n, double* A, double* evals, const char* what) {
  if (n > 0x7fffffffLL) return fail(c, QSGW_ERR_UNSUPPORTED, "%s: n too large for rocSOLVER", what);
  double* E = nullptr;
  CHECK(ws_get(c, W_EIGE, (size_t)n, &E));
  int* flags = nullptr;
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  rocblas_status st = rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_upper,
                                       (rocblas_int)n, A, (rocblas_int)n, evals, E,
                                       (rocblas_int*)(flags + 1));
  if (st != rocblas_status_success)
    return fail(c, QSGW_ERR_SOLVER, "%s: rocsolver_dsyevd status %d", what, (int)st);
  int info = 0;
  CHECK(read_flag(c, flags + 1, &info));
  if (info != 0) return fail(c, QSGW_ERR_SOLVER, "%s: dsyevd info = %d", what, info);
  return QSGW_OK;
}

// Casida eigenproblems: the two-stage solver from this size on (QSGW_EIG_AUTO).
constexpr int64_t kEigTwoStageMin = 8192;
inline bool eig_two_stage_for(const qsgw_ctx* c, int64_t n) {
  return c->eig_solver == QSGW_EIG_TWO_STAGE ||
         (c->eig_solver == QSGW_EIG_AUTO && n >= kEigTwoStageMin);
}
inline int eig_casida(qsgw_ctx* c, int64_t n, double* A, double* evals, const char* what) {
  if (eig_two_stage_for(c, n)) return eig_two_stage(c, n, A, evals, what);
  return syevd(c, n, A, evals, what);
}

// V (+)= 1/2 (G + G^T), G = sum of the nz partial slices of part.  Long sums
// go through a first level of 32 slices per group (coalesced reads, many
// threads), then the symmetric sum over the group results.
inline int reduce_sym(qsgw_ctx* c, const double* part, int64_t nz, int64_t n, double* V, int accumulate) {
  const int64_t nn = n * n;
  constexpr int64_t zg = 32;
  if (nz > 2 * zg) {
    const int64_t ng = (nz + zg - 1) / zg;
    double* red = nullptr;
    CHECK(ws_get(c, W_REDPART, (size_t)(ng * nn), &red));
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks_for(ng * nn)), dim3(256), 0, c->stream, part, nz,
                       nn, zg, red);
    CHECK(launch_check(c, "k_sum_slices"));
    part = red;
    nz = ng;
  }
  hipLaunchKernelGGL(k_reduce_sym, dim3(blocks_for(nn)), dim3(256), 0, c->stream, part, nz, n, V,
                     accumulate);
  return launch_check(c, "k_reduce_sym");
}

// Finite-input check of an entry point: one pass over each input array on
// the device (a NaN or infinity sets that array's bit), then one read-back.
struct FiniteArg {
  const void* p;
  int64_t n;
  const char* name;
  bool f32;
};
inline FiniteArg fin(const double* p, int64_t n, const char* name) { return {p, n, name, false}; }
inline FiniteArg fin32(const float* p, int64_t n, const char* name) { return {p, n, name, true}; }

inline int check_finite(qsgw_ctx* c, const char* what, std::initializer_list<FiniteArg> args) {
  int* flags = nullptr;
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  int* bad = flags + 5;
  HIP_TRY(c, hipMemsetAsync(bad, 0, sizeof(int), c->stream));
  int bit = 0;
  for (const FiniteArg& a : args) {
    if (a.p && a.n > 0) {
      int64_t nb = (a.n + 255) / 256;
      const unsigned grid = (unsigned)(nb < 2048 ? nb : 2048);
      if (a.f32)
        hipLaunchKernelGGL(k_check_finite_f32, dim3(grid), dim3(256), 0, c->stream,
                           static_cast<const float*>(a.p), a.n, bad, 1 << bit);
      else
        hipLaunchKernelGGL(k_check_finite, dim3(grid), dim3(256), 0, c->stream,
                           static_cast<const double*>(a.p), a.n, bad, 1 << bit);
    }
    ++bit;
  }
  CHECK(launch_check(c, "k_check_finite"));
  int mask = 0;
  CHECK(read_flag(c, bad, &mask));
  if (mask) {
    int i = 0;
    for (const FiniteArg& a : args) {
      if (mask & (1 << i)) return fail(c, QSGW_ERR_NONFINITE, "%s: non-finite value in %s", what, a.name);
      ++i;
    }
  }
  return QSGW_OK;
}

inline int check_common(qsgw_ctx* c, int64_t nbf, int64_t naux) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (nbf < 1 || naux < 1) return fail(c, QSGW_ERR_INVALID_ARG, "need nbf >= 1 and naux >= 1");
  if (nbf > 46340) return fail(c, QSGW_ERR_INVALID_ARG, "nbf too large");
  return QSGW_OK;
}

inline int single_begin(qsgw_ctx* c, int stage) {
  c->last_stage = stage;
  return record(c, 0);
}
inline int single_end(qsgw_ctx* c) { return record(c, 1); }

}  // namespace
