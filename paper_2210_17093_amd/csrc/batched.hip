// Batched qsGW iterations: many independent molecules of different sizes,
// one launch per stage over all of them.
//
// Every molecule keeps the single-problem algorithm (same tile shapes, K-split
// plans and epilogues, so its arithmetic is that of qsgw_iterate); the batch
// dimension is added by
//   * grouped GEMM launches: a device table with one job per molecule (its
//     operands, sizes and split plan); a workgroup finds its job by binary
//     search over the jobs' first workgroup ids (gemm_grouped_kernel);
//   * segment kernels for the element-wise steps: the per-molecule element
//     counts are prefix-summed and a thread finds its molecule by binary
//     search;
//   * rocSOLVER strided-batched dsyevd per size bucket for the Casida and Fock
//     eigenproblems.  A matrix of order n in a bucket of order nb is stored
//     nb x nb with zero coupling to the padding and padding diagonal above the
//     Gershgorin bound of the matrix, so its n lowest eigenpairs are its own.
// With QSGW_OPT_GRAPH the kernel segments between the eigensolves are
// captured into hipGraphs during the first iteration and replayed after it.
#include "internal.hpp"

#include <algorithm>
#include <map>

namespace {

// ------------------------------------------------------------ descriptors --
struct Mol {
  int64_t nbf, naux, nocc, nv, ntr, nn;
  int64_t nbM, nbF;  // padded eigenproblem orders (bucket sizes)
  const double* B_ao;
  const double* h;
  double* eps;  // state
  double* C;    // state
  double *T, *Bmo, *Bt, *delta, *sqd, *M, *Mev, *rho, *rhopart, *w, *wh, *part, *V, *hmo, *J,
      *tmp, *tmp2, *F, *Fev, *Cn, *cp;
  double* Vc;     // state: AO-basis potential, or null
  double* diag;   // state: per-state diagonal outputs [nbf][4], or null
  int64_t* itc;   // iterations done (device copy of the state's counter)
  int64_t rho_nz;
  const int32_t* pblocks;
  int64_t npblocks;
  double eta;
  double* deps;  // this molecule's max |d eps| slot
  double* pad;   // [0] Casida padding diagonal, [1] Fock padding diagonal
  int* flag;
};

enum Seg { S_NTR = 0, S_NAUXNTR, S_NN, S_NBM2, S_NBF2, S_NAUX, S_NBF, S_CHM, S_CHF, S_COUNT };
constexpr int64_t kGerCols = 256;  // columns per Gershgorin workgroup

__device__ __forceinline__ int64_t seg_find(const int64_t* pre, int64_t n, int64_t idx) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= idx) lo = mid; else hi = mid - 1;
  }
  return lo;
}

#define SEG_PROLOGUE(total)                                                          \
  const int64_t gidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;               \
  if (gidx >= (total)) return;                                                       \
  const int64_t mi = seg_find(pre, nmol, gidx);                                      \
  const Mol& m = mols[mi];                                                           \
  const int64_t li = gidx - pre[mi];

// ---------------------------------------------------------- segment kernels --
__global__ void kb_zero_flags(const Mol* mols, int64_t nmol) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nmol) *mols[i].flag = 0;
}

__global__ void kb_transitions(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  const int64_t i = li / m.nv, a = m.nocc + (li - (li / m.nv) * m.nv);
  const double d = m.eps[a] - m.eps[i];
  if (!(d > 0.0) || !isfinite(d)) atomicOr(m.flag, 1);
  m.delta[li] = d;
  m.sqd[li] = sqrt(d > 0.0 ? d : 0.0);
}

__global__ void kb_gather_bia(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  const int64_t P = li / m.ntr, t = li - (li / m.ntr) * m.ntr;
  const int64_t i = t / m.nv, a = m.nocc + (t - (t / m.nv) * m.nv);
  m.Bt[li] = m.Bmo[(P * m.nbf + i) * m.nbf + a] * m.sqd[t];
}

// Padding diagonal = 1 + max_t sum_u |A[u][t]| over the matrix's own n x n
// block (ld = nb), the Gershgorin bound of its spectrum.  A is symmetric, so
// column sums are row sums: workgroup g of a molecule takes columns
// [256 g, 256 g + 256), one per thread (consecutive threads read consecutive
// addresses), and writes the largest sum to part[g]; kb_gershgorin_max then
// takes the largest over the molecule's workgroups.  which = 0 Casida, 1 Fock.
__global__ void kb_gershgorin(const Mol* mols, const int64_t* pre, int64_t nmol, int which,
                              double* part) {
  __shared__ double red[4];
  const int64_t g = blockIdx.x;
  const int64_t mi = seg_find(pre, nmol, g);
  const Mol& m = mols[mi];
  const double* A = which == 0 ? m.M : m.F;
  const int64_t n = which == 0 ? m.ntr : m.nbf, nb = which == 0 ? m.nbM : m.nbF;
  const int64_t t = (g - pre[mi]) * kGerCols + threadIdx.x;
  double best = 0.0;
  if (t < n) {
    double s = 0.0;
    for (int64_t u = 0; u < n; ++u) s += fabs(A[u * nb + t]);
    best = s;
  }
  for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_down(best, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, red[k]);
    part[g] = r;
  }
}

__global__ void kb_gershgorin_max(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total,
                                  int which, const double* part) {
  const int64_t mi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (mi >= nmol) return;
  const int64_t g1 = mi + 1 < nmol ? pre[mi + 1] : total;
  double r = 0.0;
  for (int64_t g = pre[mi]; g < g1; ++g) r = fmax(r, part[g]);
  mols[mi].pad[which] = 1.0 + r;
}

// Padding of the nb x nb storage outside the matrix's own n x n block.
__global__ void kb_pad(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total,
                       int which) {
  SEG_PROLOGUE(total)
  const int64_t n = which == 0 ? m.ntr : m.nbf, nb = which == 0 ? m.nbM : m.nbF;
  const int64_t t = li / nb, u = li - (li / nb) * nb;
  if (t < n && u < n) return;
  double* A = which == 0 ? m.M : m.F;
  A[li] = (t == u) ? m.pad[which] : 0.0;
}

__global__ void kb_omega(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  const double l = m.Mev[li];
  if (!(l > 0.0) || !isfinite(l)) atomicOr(m.flag, 2);
  m.Mev[li] = sqrt(l > 0.0 ? l : 0.0);
}

__global__ void kb_rho_reduce(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  const int64_t len = m.naux * m.ntr;
  double v = 0.0;
  for (int64_t z = 0; z < m.rho_nz; ++z) v += m.rhopart[z * len + li];
  m.rho[li] = v * sqrt(2.0 / m.Mev[li - (li / m.ntr) * m.ntr]);
}

// which = 0: V = 1/2 (sum_z part + transpose) (qsGW matrix);
// which = 1: F = sym(hmo) + J - sum_z part + V  (Fock, into padded storage).
__global__ void kb_reduce_nn(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total,
                             const int64_t* nz, int which) {
  SEG_PROLOGUE(total)
  const int64_t n = m.nbf, r = li / n, c = li - (li / n) * n, nn = m.nn;
  const int64_t z1 = nz[mi];
  if (which == 0) {
    double a = 0.0, b = 0.0;
    for (int64_t z = 0; z < z1; ++z) {
      a += m.part[z * nn + r * n + c];
      b += m.part[z * nn + c * n + r];
    }
    m.V[li] = 0.5 * (a + b);
  } else {
    double k = 0.0;
    for (int64_t z = 0; z < z1; ++z) k += m.part[z * nn + li];
    const double hv = 0.5 * (m.hmo[r * n + c] + m.hmo[c * n + r]);
    m.F[r * m.nbF + c] = hv + m.J[li] - k + m.V[li];
  }
}

__global__ void kb_occ_trace(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  double s = 0.0;
  for (int64_t i = 0; i < m.nocc; ++i) s += m.Bmo[(li * m.nbf + i) * m.nbf + i];
  m.cp[li] = s;
}

__global__ void kb_hartree(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  double s = 0.0;
  for (int64_t P = 0; P < m.naux; ++P) s += m.cp[P] * m.Bmo[P * m.nn + li];
  m.J[li] = 2.0 * s;
}

__global__ void kb_fix_signs(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  const int64_t n = m.nbf, j = li;
  double best = -1.0, val = 1.0;
  for (int64_t r = 0; r < n; ++r) {
    const double x = m.Cn[r * n + j];
    if (fabs(x) > best) {
      best = fabs(x);
      val = x;
    }
  }
  if (val < 0.0)
    for (int64_t r = 0; r < n; ++r) m.Cn[r * n + j] = -m.Cn[r * n + j];
}

// One workgroup per molecule: max |eps' - eps| (eps' = first nbf Fock eigenvalues).
__global__ void kb_deps(const Mol* mols) {
  __shared__ double red[4];
  const Mol& m = mols[blockIdx.x];
  double best = 0.0;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < m.nbf; i += blockDim.x) {
    const double d = fabs(m.Fev[i] - m.eps[i]);
    if (!isfinite(d)) bad = true;
    best = fmax(best, d);
  }
  if (bad) best = INFINITY;
  for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_down(best, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, red[k]);
    *m.deps = r;
  }
}

// State update: C <- C', eps <- eps' (nbf x nbf + nbf elements per molecule).
__global__ void kb_commit(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  m.C[li] = m.Cn[li];
  if (li < m.nbf) m.eps[li] = m.Fev[li];
  if (li == 0) *m.itc += 1;
}

// Potential mixing in the AO basis (molecules with a Vc buffer), after
// tmp2 = C V C^T:
//   kb_mix_a: tmp = mix tmp2 + (1 - mix) Vc   (mixing: mix != 1 and an earlier iteration)
//             tmp = tmp2                      (otherwise)
//   kb_mix_b: Vc = 1/2 (tmp + tmp^T)
//   kb_mix_c: V = 1/2 (tmp2 + tmp2^T) with tmp2 = C^T Vc C   (mixing only)
__device__ __forceinline__ bool mixing(const Mol& m, double mix) {
  return mix != 1.0 && *m.itc > 0;
}

__global__ void kb_mix_a(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total,
                         double mix) {
  SEG_PROLOGUE(total)
  if (!m.Vc) return;
  m.tmp[li] = mixing(m, mix) ? mix * m.tmp2[li] + (1.0 - mix) * m.Vc[li] : m.tmp2[li];
}

__global__ void kb_mix_b(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total) {
  SEG_PROLOGUE(total)
  if (!m.Vc) return;
  const int64_t n = m.nbf, r = li / n, c = li - (li / n) * n;
  m.Vc[li] = 0.5 * (m.tmp[r * n + c] + m.tmp[c * n + r]);
}

__global__ void kb_mix_c(const Mol* mols, const int64_t* pre, int64_t nmol, int64_t total,
                         double mix) {
  SEG_PROLOGUE(total)
  if (!m.Vc || !mixing(m, mix)) return;
  const int64_t n = m.nbf, r = li / n, c = li - (li / n) * n;
  m.V[li] = 0.5 * (m.tmp2[r * n + c] + m.tmp2[c * n + r]);
}

// Per-state diagonal outputs (one workgroup per state of every molecule with
// a diag buffer): Eq. (17) at omega = eps_m and its derivative from the
// residues of all excitations, and the exchange diagonal.
__global__ void kb_diag(const Mol* mols, const int64_t* pre, int64_t nmol) {
  const int64_t idx = blockIdx.x;
  const int64_t mi = seg_find(pre, nmol, idx);
  const Mol& m = mols[mi];
  const int64_t st = idx - pre[mi];
  if (!m.diag || st >= m.nbf) return;
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  diag_self_partial(m.w + st * m.nbf * m.ntr, m.eps, m.Mev, st, m.nbf, m.nocc, m.ntr, m.eta, r);
  r[3] = exchange_diag_partial(m.Bmo, m.naux, m.nbf, m.nocc, st);
  block_sum<4>(r);
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) m.diag[st * 4 + q] = r[q];
}

// ------------------------------------------------------------- host side --
struct Bucket {
  int64_t nb = 0;
  std::vector<int64_t> mols;  // molecule indices
  double* A = nullptr;        // first matrix of the bucket
  double* ev = nullptr;       // first eigenvalue vector
  double* E = nullptr;        // dsyevd off-diagonal workspace
  int* info = nullptr;
};

struct Plan {
  std::vector<Mol> mols;
  Mol* dmols = nullptr;
  int64_t* dpre[S_COUNT] = {};
  int64_t total[S_COUNT] = {};
  int64_t* sig_nz = nullptr;   // device, per molecule
  int64_t* exc_nz = nullptr;   // device, per molecule
  std::vector<Bucket> bM, bF;
  double* deps = nullptr;      // device [nmol]
  double* gpart = nullptr;     // device, Gershgorin partial maxima (one per workgroup)
  double mix = 1.0;
};

template <class J>
int upload_jobs(qsgw_ctx* c, std::vector<J>& jobs, int bm, int bn, char*& cursor, const J** out,
                int64_t* nwg) {
  int64_t wg = 0;
  for (auto& j : jobs) {
    if (!loader_offsets_fit(j.a, bm) || !loader_offsets_fit(j.b, bn))
      return fail(c, QSGW_ERR_UNSUPPORTED, "batched: operand strides too large for the tile loader");
    j.wg_begin = wg;
    const int64_t tiles = j.tiles_n > 0 ? j.tiles_m * j.tiles_n : j.tiles_m * (j.tiles_m + 1) / 2;
    const int64_t nz = (j.K + j.kchunk - 1) / j.kchunk;
    wg += tiles * j.nbatch * nz;
  }
  const size_t bytes = jobs.size() * sizeof(J);
  HIP_TRY(c, hipMemcpyAsync(cursor, jobs.data(), bytes, hipMemcpyHostToDevice, c->stream));
  *out = reinterpret_cast<const J*>(cursor);
  cursor += (bytes + 255) / 256 * 256;
  *nwg = wg;
  return QSGW_OK;
}

template <class J>
size_t job_bytes(size_t n) {
  return (n * sizeof(J) + 255) / 256 * 256;
}

// Job of one molecule: tiles_n = 0 marks a symmetric (upper-tile) problem.
template <class OA, class OB, class EPI>
GemmJob<OA, OB, EPI> job(OA a, OB b, EPI e, int64_t M, int64_t N, int64_t K, int64_t nbatch,
                         int BM, int BN, SplitPlan sp, bool tri) {
  GemmJob<OA, OB, EPI> j{a, b, e, M, N, K, sp.nz > 1 ? sp.kchunk : K, (M + BM - 1) / BM,
                         tri ? 0 : (N + BN - 1) / BN, nbatch, 0};
  return j;
}

constexpr int64_t kComputeUnits = 256;

template <int BM, int BN, bool TRI, class CT, class OA, class OB, class EPI>
int launch_grouped(qsgw_ctx* c, const char* what, const GemmJob<OA, OB, EPI>* jobs, int64_t njobs,
                   int64_t nwg) {
  if (nwg <= 0) return QSGW_OK;
  if (nwg > 0x7fffffffLL) return fail(c, QSGW_ERR_INVALID_ARG, "%s: launch too large", what);
  int64_t grid = nwg;
  if (c->tiles.persistent > 0 && grid > c->tiles.persistent * kComputeUnits)
    grid = c->tiles.persistent * kComputeUnits;
  // (the split-BF16 products take k tiles of 32, one BF16 instruction's depth)
  constexpr int BK = is_bf16x3<CT>::value ? 32 : 16;
  hipLaunchKernelGGL((gemm_grouped_kernel<BM, BN, OA, OB, EPI, TRI, BK, CT>), dim3((unsigned)grid),
                     dim3(256), 0, c->stream, jobs, njobs, nwg);
  return launch_check(c, what);
}

// Grouped launch with the tile shape chosen at run time.
template <bool TRI, class CT, class OA, class OB, class EPI>
int launch_shape(qsgw_ctx* c, int shape, const char* what, const GemmJob<OA, OB, EPI>* jobs,
                 int64_t njobs, int64_t nwg) {
  switch (shape) {
    case SH_64x64:
      return launch_grouped<64, 64, TRI, CT>(c, what, jobs, njobs, nwg);
    case SH_128x128:
      return launch_grouped<128, 128, TRI, CT>(c, what, jobs, njobs, nwg);
    default:
      if constexpr (TRI) {
        return fail(c, QSGW_ERR_INVALID_ARG, "%s: symmetric products take square tiles", what);
      } else {
        return launch_grouped<128, 64, false, CT>(c, what, jobs, njobs, nwg);
      }
  }
}

// The kernel body handles a symmetric job through tiles_n = 0: the grouped
// kernel is instantiated with TRI and reads tiles_m only.
typedef GemmJob<Strided<true>, Strided<false>, EpiStore> JobTF;
typedef GemmJob<Strided<false>, Strided<false>, EpiStore> JobFF;
typedef GemmJob<Strided<false>, Strided<false>, EpiCasida> JobCas;
typedef GemmJob<Strided<true>, Strided<true>, EpiStore> JobTT;
typedef GemmJob<PairRows<8, 16>, Strided<false>, EpiPairResidue> JobW;
typedef GemmJob<OccRowsOp, OccRowsOp, EpiStore> JobK;

struct Jobs {
  const JobTF* mo1; int64_t mo1_wg;
  const JobFF* mo2; int64_t mo2_wg;
  const JobCas* cas; int64_t cas_wg;
  const JobTT* rho; int64_t rho_wg;
  const JobW* w; int64_t w_wg;
  const JobTT* sig; int64_t sig_wg;
  const JobTF* hc1; int64_t hc1_wg;   // tmp = h C
  const JobFF* hc2; int64_t hc2_wg;   // hmo = C^T tmp
  const JobK* exc; int64_t exc_wg;
  const JobTT* rot; int64_t rot_wg;   // C' = C U
  int64_t n;
  // potential of molecules with a Vc buffer (nv of them): tmp2 = C V C^T,
  // and with mixing (nmix of them) tmp2 = C^T Vc C
  const JobTF* cg3; int64_t cg3_wg;   // tmp = C V
  const JobTT* cg4; int64_t cg4_wg;   // tmp2 = tmp C^T
  const JobTF* ct1; int64_t ct1_wg;   // tmp = Vc C
  const JobFF* ct2; int64_t ct2_wg;   // tmp2 = C^T tmp
  int64_t nv, nmix;
};

// CTM: arithmetic of the MO transform, CT: of the Casida build (split-BF16
// keeps the MO transform on the FP32 matrix cores, as the single path does)
template <class CTM, class CT>
int segment_a(qsgw_ctx* c, Plan& P, const Jobs& J, Spans* sp) {
  const int64_t nmol = (int64_t)P.mols.size();
  hipLaunchKernelGGL(kb_zero_flags, dim3(blocks_for(nmol)), dim3(256), 0, c->stream, P.dmols, nmol);
  SPAN_OPEN(sp, kKMo1);
  CHECK((launch_shape<false, CTM>(c, c->tiles.shape[TU_MO1], "batched mo/1", J.mo1, J.n, J.mo1_wg)));
  SPAN_CLOSE(sp);
  SPAN_OPEN(sp, kKMo2);
  CHECK((launch_shape<true, CTM>(c, c->tiles.shape[TU_MO2], "batched mo/2", J.mo2, J.n, J.mo2_wg)));
  SPAN_CLOSE(sp);
  SPAN_OPEN(sp, kKCasida);
  hipLaunchKernelGGL(kb_transitions, dim3(blocks_for(P.total[S_NTR])), dim3(256), 0, c->stream,
                     P.dmols, P.dpre[S_NTR], nmol, P.total[S_NTR]);
  hipLaunchKernelGGL(kb_gather_bia, dim3(blocks_for(P.total[S_NAUXNTR])), dim3(256), 0, c->stream,
                     P.dmols, P.dpre[S_NAUXNTR], nmol, P.total[S_NAUXNTR]);
  CHECK((launch_shape<true, CT>(c, c->tiles.shape[TU_CASIDA], "batched casida", J.cas, J.n,
                                J.cas_wg)));
  SPAN_CLOSE(sp);
  hipLaunchKernelGGL(kb_gershgorin, dim3((unsigned)P.total[S_CHM]), dim3(kGerCols), 0, c->stream,
                     P.dmols, P.dpre[S_CHM], nmol, 0, P.gpart);
  hipLaunchKernelGGL(kb_gershgorin_max, dim3(blocks_for(nmol)), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_CHM], nmol, P.total[S_CHM], 0, P.gpart);
  hipLaunchKernelGGL(kb_pad, dim3(blocks_for(P.total[S_NBM2])), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_NBM2], nmol, P.total[S_NBM2], 0);
  return launch_check(c, "batched segment A");
}

template <class CT>
int segment_b(qsgw_ctx* c, Plan& P, const Jobs& J, Spans* sp) {
  const int64_t nmol = (int64_t)P.mols.size();
  SPAN_OPEN(sp, kKRho);
  hipLaunchKernelGGL(kb_omega, dim3(blocks_for(P.total[S_NTR])), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_NTR], nmol, P.total[S_NTR]);
  CHECK((launch_shape<false, CT>(c, c->tiles.shape[TU_RHO], "batched rho", J.rho, J.n, J.rho_wg)));
  hipLaunchKernelGGL(kb_rho_reduce, dim3(blocks_for(P.total[S_NAUXNTR])), dim3(256), 0, c->stream,
                     P.dmols, P.dpre[S_NAUXNTR], nmol, P.total[S_NAUXNTR]);
  SPAN_CLOSE(sp);
  SPAN_OPEN(sp, kKW);
  CHECK((launch_grouped<128, 128, false, CT>(c, "batched residues", J.w, J.n, J.w_wg)));
  SPAN_CLOSE(sp);
  return launch_check(c, "batched segment B1");
}

int segment_b2(qsgw_ctx* c, Plan& P, const Jobs& J, Spans* sp) {
  const int64_t nmol = (int64_t)P.mols.size();
  SPAN_OPEN(sp, kKSigma);
  CHECK((launch_shape<false, double>(c, c->tiles.shape[TU_SIGMA], "batched sigma", J.sig, J.n,
                                     J.sig_wg)));
  SPAN_CLOSE(sp);
  SPAN_OPEN(sp, kKSigmaRed);
  hipLaunchKernelGGL(kb_reduce_nn, dim3(blocks_for(P.total[S_NN])), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_NN], nmol, P.total[S_NN], P.sig_nz, 0);
  SPAN_CLOSE(sp);
  SPAN_OPEN(sp, kKFock);
  if (J.nv > 0) {
    CHECK((launch_grouped<64, 64, false, double>(c, "batched C V", J.cg3, J.nv, J.cg3_wg)));
    CHECK((launch_grouped<64, 64, false, double>(c, "batched C V C^T", J.cg4, J.nv, J.cg4_wg)));
    hipLaunchKernelGGL(kb_mix_a, dim3(blocks_for(P.total[S_NN])), dim3(256), 0, c->stream, P.dmols,
                       P.dpre[S_NN], nmol, P.total[S_NN], P.mix);
    hipLaunchKernelGGL(kb_mix_b, dim3(blocks_for(P.total[S_NN])), dim3(256), 0, c->stream, P.dmols,
                       P.dpre[S_NN], nmol, P.total[S_NN]);
    if (J.nmix > 0) {
      CHECK((launch_grouped<64, 64, false, double>(c, "batched Vc C", J.ct1, J.nmix, J.ct1_wg)));
      CHECK((launch_grouped<64, 64, false, double>(c, "batched C^T Vc C", J.ct2, J.nmix, J.ct2_wg)));
      hipLaunchKernelGGL(kb_mix_c, dim3(blocks_for(P.total[S_NN])), dim3(256), 0, c->stream,
                         P.dmols, P.dpre[S_NN], nmol, P.total[S_NN], P.mix);
    }
  }
  CHECK((launch_grouped<64, 64, false, double>(c, "batched hC", J.hc1, J.n, J.hc1_wg)));
  CHECK((launch_grouped<64, 64, false, double>(c, "batched C^T hC", J.hc2, J.n, J.hc2_wg)));
  hipLaunchKernelGGL(kb_occ_trace, dim3(blocks_for(P.total[S_NAUX])), dim3(256), 0, c->stream,
                     P.dmols, P.dpre[S_NAUX], nmol, P.total[S_NAUX]);
  hipLaunchKernelGGL(kb_hartree, dim3(blocks_for(P.total[S_NN])), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_NN], nmol, P.total[S_NN]);
  CHECK((launch_shape<true, double>(c, c->tiles.shape[TU_EXCHANGE], "batched exchange", J.exc, J.n,
                                    J.exc_wg)));
  hipLaunchKernelGGL(kb_reduce_nn, dim3(blocks_for(P.total[S_NN])), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_NN], nmol, P.total[S_NN], P.exc_nz, 1);
  SPAN_CLOSE(sp);
  hipLaunchKernelGGL(kb_gershgorin, dim3((unsigned)P.total[S_CHF]), dim3(kGerCols), 0, c->stream,
                     P.dmols, P.dpre[S_CHF], nmol, 1, P.gpart);
  hipLaunchKernelGGL(kb_gershgorin_max, dim3(blocks_for(nmol)), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_CHF], nmol, P.total[S_CHF], 1, P.gpart);
  hipLaunchKernelGGL(kb_pad, dim3(blocks_for(P.total[S_NBF2])), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_NBF2], nmol, P.total[S_NBF2], 1);
  return launch_check(c, "batched segment B2");
}

int segment_c(qsgw_ctx* c, Plan& P, const Jobs& J, Spans* sp) {
  const int64_t nmol = (int64_t)P.mols.size();
  CHECK((launch_grouped<64, 64, false, double>(c, "batched rotate", J.rot, J.n, J.rot_wg)));
  hipLaunchKernelGGL(kb_fix_signs, dim3(blocks_for(P.total[S_NBF])), dim3(256), 0, c->stream,
                     P.dmols, P.dpre[S_NBF], nmol, P.total[S_NBF]);
  hipLaunchKernelGGL(kb_deps, dim3((unsigned)nmol), dim3(256), 0, c->stream, P.dmols);
  hipLaunchKernelGGL(kb_commit, dim3(blocks_for(P.total[S_NN])), dim3(256), 0, c->stream, P.dmols,
                     P.dpre[S_NN], nmol, P.total[S_NN]);
  return launch_check(c, "batched segment C");
}

int aux_streams(qsgw_ctx* c) {
  if (c->aux_ready) return QSGW_OK;
  for (int i = 0; i < qsgw_ctx::kAux; ++i) {
    if (!c->aux[i]) HIP_TRY(c, hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking));
    if (!c->join[i]) HIP_TRY(c, hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming));
    if (!c->aux_blas[i]) {
      if (rocblas_create_handle(&c->aux_blas[i]) != rocblas_status_success) {
        c->aux_blas[i] = nullptr;
        return fail(c, QSGW_ERR_SOLVER, "rocblas_create_handle failed");
      }
      if (rocblas_set_stream(c->aux_blas[i], c->aux[i]) != rocblas_status_success)
        return fail(c, QSGW_ERR_SOLVER, "rocblas_set_stream failed");
    }
  }
  if (!c->fork) HIP_TRY(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
  c->aux_ready = true;
  return QSGW_OK;
}

// Strided-batched dsyevd per bucket; the buckets (largest first) go
// round-robin over the context stream and the auxiliary streams, which fork
// from and join back into the context stream.
int eig_buckets(qsgw_ctx* c, std::vector<Bucket>& bs) {
  CHECK(aux_streams(c));
  std::vector<Bucket*> order;
  for (auto& b : bs) order.push_back(&b);
  std::sort(order.begin(), order.end(), [](const Bucket* a, const Bucket* b) {
    return a->nb * a->nb * (int64_t)a->mols.size() > b->nb * b->nb * (int64_t)b->mols.size();
  });
  const int lanes = 1 + qsgw_ctx::kAux;
  HIP_TRY(c, hipEventRecord(c->fork, c->stream));
  for (int i = 0; i < qsgw_ctx::kAux; ++i) HIP_TRY(c, hipStreamWaitEvent(c->aux[i], c->fork, 0));
  for (size_t j = 0; j < order.size(); ++j) {
    Bucket& b = *order[j];
    const int lane = (int)(j % lanes);
    rocblas_handle h = lane == 0 ? c->blas : c->aux_blas[lane - 1];
    const rocblas_stride sA = (rocblas_stride)(b.nb * b.nb), sD = (rocblas_stride)b.nb;
    rocblas_status st = rocsolver_dsyevd_strided_batched(
        h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)b.nb, b.A, (rocblas_int)b.nb,
        sA, b.ev, sD, b.E, sD, (rocblas_int*)b.info, (rocblas_int)b.mols.size());
    if (st != rocblas_status_success)
      return fail(c, QSGW_ERR_SOLVER, "rocsolver_dsyevd_strided_batched status %d (n = %lld)",
                  (int)st, (long long)b.nb);
  }
  for (int i = 0; i < qsgw_ctx::kAux; ++i) {
    HIP_TRY(c, hipEventRecord(c->join[i], c->aux[i]));
    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->join[i], 0));
  }
  return QSGW_OK;
}

struct Graphs {
  hipGraphExec_t x[4] = {nullptr, nullptr, nullptr, nullptr};
  ~Graphs() {
    for (auto g : x)
      if (g) (void)hipGraphExecDestroy(g);
  }
};

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

}  // namespace

extern "C" int qsgw_iterate_batched(qsgw_ctx* c, int64_t nmol, const qsgw_problem* probs,
                                    qsgw_state* states, const qsgw_options* o,
                                    qsgw_report* reports) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (nmol < 1 || !probs || !states || !o) return fail(c, QSGW_ERR_INVALID_ARG, "bad arguments");
  if (o->precision != QSGW_PREC_FP64 && o->precision != QSGW_PREC_FP32 &&
      o->precision != QSGW_PREC_SPLIT_BF16)
    return fail(c, QSGW_ERR_UNSUPPORTED, "precision %d is not available", o->precision);
  if (!(o->eta > 0.0) || !isfinite(o->eta)) return fail(c, QSGW_ERR_INVALID_ARG, "need eta > 0");
  if (o->max_iter < 1) return fail(c, QSGW_ERR_INVALID_ARG, "need max_iter >= 1");
  if (!(o->mix > 0.0 && o->mix <= 1.0)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < mix <= 1");
  if (o->s_block != 0)
    return fail(c, QSGW_ERR_UNSUPPORTED, "the batched iteration keeps every excitation resident");
  if (o->fock_mode != QSGW_FOCK_FULL_JK)
    return fail(c, QSGW_ERR_UNSUPPORTED, "fock_mode %d is not available", o->fock_mode);
  if (o->warm_start)
    return fail(c, QSGW_ERR_UNSUPPORTED, "warm_start: apply qsgw_warm_start to each molecule");
  if (o->diis != 0)
    return fail(c, QSGW_ERR_UNSUPPORTED, "diis: qsgw_iterate only");
  if (o->flags & ~(int64_t)QSGW_OPT_GRAPH)
    return fail(c, QSGW_ERR_UNSUPPORTED, "flags other than QSGW_OPT_GRAPH");
  // reduced precision: FP32 or split-BF16 products (FP32 accumulation, each
  // workgroup's k range bounded as in the single path)
  const bool fp32 = o->precision != QSGW_PREC_FP64;
  const bool x3 = o->precision == QSGW_PREC_SPLIT_BF16;

  // ------------------------------------------------------------ layout --
  Plan P;
  P.mols.resize(nmol);
  std::map<int64_t, std::vector<int64_t>> bucketM, bucketF;
  size_t nd = 0, ni = 0;  // doubles and int32 of workspace
  std::vector<std::vector<int32_t>> tables(nmol);
  std::vector<int64_t> sig_nz(nmol), exc_nz(nmol);
  for (int64_t i = 0; i < nmol; ++i) {
    const qsgw_problem& p = probs[i];
    Mol& m = P.mols[i];
    m.nbf = p.nbf;
    m.naux = p.naux;
    m.nocc = p.nocc;
    if (!(m.nocc > 0 && m.nocc < m.nbf) || m.naux < 1 || m.nbf > 4096)
      return fail(c, QSGW_ERR_INVALID_ARG, "molecule %lld: need 0 < nocc < nbf <= 4096, naux >= 1",
                  (long long)i);
    if (!p.B_ao || !p.h || !states[i].eps || !states[i].C)
      return fail(c, QSGW_ERR_INVALID_ARG, "molecule %lld: null pointer", (long long)i);
    if (o->mix != 1.0 && !states[i].Vc)
      return fail(c, QSGW_ERR_INVALID_ARG, "molecule %lld: mixing needs a Vc buffer", (long long)i);
    if (states[i].iteration < 0)
      return fail(c, QSGW_ERR_INVALID_ARG, "molecule %lld: negative iteration count", (long long)i);
    m.nv = m.nbf - m.nocc;
    m.ntr = m.nocc * m.nv;
    m.nn = m.nbf * m.nbf;
    m.nbM = round_up(m.ntr, 128);
    m.nbF = round_up(m.nbf, 32);
    m.B_ao = p.B_ao;
    m.h = p.h;
    m.eps = states[i].eps;
    m.C = states[i].C;
    m.Vc = states[i].Vc;
    m.diag = states[i].diag;
    m.eta = o->eta;
    bucketM[m.nbM].push_back(i);
    bucketF[m.nbF].push_back(i);
    const SplitPlan rs = rho_split(c->tiles, m.naux, m.ntr, m.ntr, fp32 ? kFp32MaxK : m.ntr);
    m.rho_nz = rs.nz;
    sig_nz[i] = sigma_split(c->tiles, m.nbf, m.ntr).nz;
    exc_nz[i] = exchange_split(c->tiles, m.nbf, m.naux, m.nocc).nz;
    const int64_t pnz = std::max(sig_nz[i], exc_nz[i]);
    nd += 2 * m.naux * m.nn + m.naux * m.ntr * (2 + m.rho_nz) + 2 * m.ntr + 2 * m.nn * m.ntr +
          pnz * m.nn + 7 * m.nn + m.naux + 64;
    const int64_t nmb = (m.nbf + 7) / 8, nkb = (m.nbf + 15) / 16;
    for (int64_t mb = 0; mb < nmb; ++mb)
      for (int64_t kb = 0; kb < nkb; ++kb)
        if (8 * mb <= 16 * kb + 15) tables[i].push_back((int32_t)((mb << 16) | kb));
    ni += tables[i].size();
  }
  {
    // finite inputs of every molecule: one pass each, one read-back
    int* flags = nullptr;
    CHECK(ws_get(c, W_FLAGS, 8, &flags));
    HIP_TRY(c, hipMemsetAsync(flags + 5, 0, sizeof(int), c->stream));
    for (int64_t i = 0; i < nmol; ++i) {
      const Mol& m = P.mols[i];
      const double* arr[4] = {m.B_ao, m.h, m.C, m.eps};
      const int64_t len[4] = {m.naux * m.nn, m.nn, m.nn, m.nbf};
      for (int k = 0; k < 4; ++k) {
        const int64_t nb = (len[k] + 255) / 256;
        hipLaunchKernelGGL(k_check_finite, dim3((unsigned)(nb < 512 ? nb : 512)), dim3(256), 0,
                           c->stream, arr[k], len[k], flags + 5, 1 << k);
      }
    }
    CHECK(launch_check(c, "k_check_finite"));
    int bad = 0;
    CHECK(read_flag(c, flags + 5, &bad));
    if (bad) {
      for (int64_t i = 0; i < nmol; ++i) {
        const Mol& m = P.mols[i];
        char what[64];
        snprintf(what, sizeof(what), "qsgw_iterate_batched, molecule %lld", (long long)i);
        CHECK(check_finite(c, what, {fin(m.B_ao, m.naux * m.nn, "B_ao"), fin(m.h, m.nn, "h"),
                                     fin(m.C, m.nn, "C"), fin(m.eps, m.nbf, "eps")}));
      }
    }
  }
  for (auto& kv : bucketM) nd += kv.second.size() * (kv.first * kv.first + 2 * kv.first);
  for (auto& kv : bucketF) nd += kv.second.size() * (kv.first * kv.first + 2 * kv.first);
  nd += nmol + 2 * nmol;  // deps, pads
  int64_t nger = 0;        // Gershgorin workgroups, Casida and Fock
  for (int64_t i = 0; i < nmol; ++i)
    nger += (P.mols[i].ntr + kGerCols - 1) / kGerCols + (P.mols[i].nbf + kGerCols - 1) / kGerCols;
  nd += nger;

  double* D = nullptr;
  int32_t* I = nullptr;
  CHECK(ws_get(c, W_BATCH_F64, nd, &D));
  CHECK(ws_get(c, W_BATCH_I32, ni + 64 * (bucketM.size() + bucketF.size()) + 4 * nmol, &I));
  double* dcur = D;
  auto take = [&](size_t n) {
    double* p = dcur;
    dcur += n;
    return p;
  };
  int32_t* icur = I;
  P.deps = take(nmol);
  double* pads = take(2 * nmol);
  P.gpart = take(nger);
  int* flags = reinterpret_cast<int*>(icur);
  icur += nmol;
  for (int64_t i = 0; i < nmol; ++i) {
    Mol& m = P.mols[i];
    m.T = take(m.naux * m.nn);
    m.Bmo = take(m.naux * m.nn);
    m.Bt = take(m.naux * m.ntr);
    m.rho = take(m.naux * m.ntr);
    m.rhopart = take(m.rho_nz * m.naux * m.ntr);
    m.delta = take(m.ntr);
    m.sqd = take(m.ntr);
    m.w = take(m.nn * m.ntr);
    m.wh = take(m.nn * m.ntr);
    m.part = take(std::max(sig_nz[i], exc_nz[i]) * m.nn);
    m.V = take(m.nn);
    m.hmo = take(m.nn);
    m.J = take(m.nn);
    m.tmp = take(m.nn);
    m.tmp2 = take(m.nn);
    m.Cn = take(m.nn);
    m.cp = take(m.naux);
    m.deps = P.deps + i;
    m.pad = pads + 2 * i;
    m.flag = flags + i;
    HIP_TRY(c, hipMemcpyAsync(icur, tables[i].data(), tables[i].size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream));
    m.pblocks = icur;
    m.npblocks = (int64_t)tables[i].size();
    icur += tables[i].size();
  }
  auto make_buckets = [&](std::map<int64_t, std::vector<int64_t>>& src, std::vector<Bucket>& dst,
                          bool casida) {
    for (auto& kv : src) {
      Bucket b;
      b.nb = kv.first;
      b.mols = kv.second;
      const int64_t cnt = (int64_t)b.mols.size(), nb = b.nb;
      b.A = take(cnt * nb * nb);
      b.ev = take(cnt * nb);
      b.E = take(cnt * nb);
      b.info = reinterpret_cast<int*>(icur);
      icur += cnt;
      for (int64_t j = 0; j < cnt; ++j) {
        Mol& m = P.mols[b.mols[j]];
        if (casida) {
          m.M = b.A + j * nb * nb;
          m.Mev = b.ev + j * nb;
        } else {
          m.F = b.A + j * nb * nb;
          m.Fev = b.ev + j * nb;
        }
      }
      dst.push_back(b);
    }
  };
  make_buckets(bucketM, P.bM, true);
  make_buckets(bucketF, P.bF, false);

  // segment prefix sums
  std::vector<int64_t> pre(S_COUNT * nmol);
  for (int s = 0; s < S_COUNT; ++s) {
    int64_t acc = 0;
    for (int64_t i = 0; i < nmol; ++i) {
      const Mol& m = P.mols[i];
      pre[s * nmol + i] = acc;
      const int64_t cnt[S_COUNT] = {m.ntr, m.naux * m.ntr, m.nn, m.nbM * m.nbM, m.nbF * m.nbF,
                                    m.naux, m.nbf, (m.ntr + kGerCols - 1) / kGerCols,
                                    (m.nbf + kGerCols - 1) / kGerCols};
      acc += cnt[s];
    }
    P.total[s] = acc;
  }
  int64_t* dpre = nullptr;
  CHECK(ws_get(c, W_BATCH_PRE, (size_t)(S_COUNT * nmol + 3 * nmol), &dpre));
  HIP_TRY(c, hipMemcpyAsync(dpre, pre.data(), pre.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                            c->stream));
  for (int s = 0; s < S_COUNT; ++s) P.dpre[s] = dpre + s * nmol;
  P.sig_nz = dpre + S_COUNT * nmol;
  P.exc_nz = P.sig_nz + nmol;
  HIP_TRY(c, hipMemcpyAsync(P.sig_nz, sig_nz.data(), nmol * sizeof(int64_t), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(P.exc_nz, exc_nz.data(), nmol * sizeof(int64_t), hipMemcpyHostToDevice,
                            c->stream));
  std::vector<int64_t> itc0(nmol);
  for (int64_t i = 0; i < nmol; ++i) {
    itc0[i] = states[i].iteration;
    P.mols[i].itc = P.exc_nz + nmol + i;
  }
  HIP_TRY(c, hipMemcpyAsync(P.exc_nz + nmol, itc0.data(), nmol * sizeof(int64_t),
                            hipMemcpyHostToDevice, c->stream));
  P.mix = o->mix;

  // ------------------------------------------------------------- jobs --
  std::vector<JobTF> mo1, hc1;
  std::vector<JobFF> mo2, hc2;
  std::vector<JobCas> cas;
  std::vector<JobTT> rho, sig, rot;
  std::vector<JobW> wj;
  std::vector<JobK> exc;
  std::vector<JobTF> cg3, ct1;
  std::vector<JobTT> cg4;
  std::vector<JobFF> ct2;
  const Tiles& tl = c->tiles;
  auto bm = [&](int t) { return shape_m(tl.shape[t]); };
  auto bn = [&](int t) { return shape_n(tl.shape[t]); };
  for (int64_t i = 0; i < nmol; ++i) {
    const Mol& m = P.mols[i];
    const int64_t nbf = m.nbf, naux = m.naux, ntr = m.ntr, nn = m.nn;
    const SplitPlan one{0, 1};
    mo1.push_back(job(Strided<true>{m.B_ao, nbf, 1, 0, naux * nbf}, Strided<false>{m.C, 1, nbf, 0, nbf},
                      EpiStore{m.T, nbf, 0, 0, 1.0}, naux * nbf, nbf, nbf, 1, bm(TU_MO1), bn(TU_MO1), one,
                      false));
    mo2.push_back(job(Strided<false>{m.C, 1, nbf, 0, nbf}, Strided<false>{m.T, 1, nbf, nn, nbf},
                      EpiStore{m.Bmo, nbf, nn, 0, 1.0}, nbf, nbf, nbf, naux, bm(TU_MO2), bn(TU_MO2), one,
                      true));
    cas.push_back(job(Strided<false>{m.Bt, 1, ntr, 0, ntr}, Strided<false>{m.Bt, 1, ntr, 0, ntr},
                      EpiCasida{m.M, m.delta, m.nbM}, ntr, ntr, naux, 1, bm(TU_CASIDA), bn(TU_CASIDA), one,
                      true));
    const SplitPlan rs = rho_split(tl, naux, ntr, ntr, fp32 ? kFp32MaxK : ntr);
    rho.push_back(job(Strided<true>{m.Bt, ntr, 1, 0, naux}, Strided<true>{m.M, m.nbM, 1, 0, ntr},
                      EpiStore{m.rhopart, ntr, 0, naux * ntr, 1.0}, naux, ntr, ntr, 1, bm(TU_RHO),
                      bn(TU_RHO), rs, false));
    wj.push_back(job(PairRows<8, 16>{m.Bmo, nn, 0, nbf, m.pblocks}, Strided<false>{m.rho, 1, ntr, 0, ntr},
                     EpiPairResidue{m.w, m.wh, m.pblocks, m.eps, m.Mev, nbf, m.nocc, ntr, o->eta},
                     m.npblocks * 128, ntr, naux, 1, 128, 128, one, false));
    sig.push_back(job(Strided<true>{m.wh, nbf * ntr, 1, 0, nbf}, Strided<true>{m.w, nbf * ntr, 1, 0, nbf},
                      EpiStore{m.part, nbf, 0, nn, 1.0}, nbf, nbf, nbf * ntr, 1, bm(TU_SIGMA),
                      bn(TU_SIGMA), sigma_split(tl, nbf, ntr), false));
    hc1.push_back(job(Strided<true>{m.h, nbf, 1, 0, nbf}, Strided<false>{m.C, 1, nbf, 0, nbf},
                      EpiStore{m.tmp, nbf, 0, 0, 1.0}, nbf, nbf, nbf, 1, 64, 64, one, false));
    hc2.push_back(job(Strided<false>{m.C, 1, nbf, 0, nbf}, Strided<false>{m.tmp, 1, nbf, 0, nbf},
                      EpiStore{m.hmo, nbf, 0, 0, 1.0}, nbf, nbf, nbf, 1, 64, 64, one, false));
    exc.push_back(job(OccRowsOp{m.Bmo, nbf, m.nocc}, OccRowsOp{m.Bmo, nbf, m.nocc},
                      EpiStore{m.part, nbf, 0, nn, 1.0}, nbf, nbf, naux * m.nocc, 1, bm(TU_EXCHANGE),
                      bn(TU_EXCHANGE), exchange_split(tl, nbf, naux, m.nocc), true));
    rot.push_back(job(Strided<true>{m.C, nbf, 1, 0, nbf}, Strided<true>{m.F, m.nbF, 1, 0, nbf},
                      EpiStore{m.Cn, nbf, 0, 0, 1.0}, nbf, nbf, nbf, 1, 64, 64, one, false));
    if (m.Vc) {
      // the congruences of the single-instance path: C V C^T, then C^T Vc C
      cg3.push_back(job(Strided<true>{m.C, nbf, 1, 0, nbf}, Strided<false>{m.V, 1, nbf, 0, nbf},
                        EpiStore{m.tmp, nbf, 0, 0, 1.0}, nbf, nbf, nbf, 1, 64, 64, one, false));
      cg4.push_back(job(Strided<true>{m.tmp, nbf, 1, 0, nbf}, Strided<true>{m.C, nbf, 1, 0, nbf},
                        EpiStore{m.tmp2, nbf, 0, 0, 1.0}, nbf, nbf, nbf, 1, 64, 64, one, false));
      if (o->mix != 1.0) {
        ct1.push_back(job(Strided<true>{m.Vc, nbf, 1, 0, nbf}, Strided<false>{m.C, 1, nbf, 0, nbf},
                          EpiStore{m.tmp, nbf, 0, 0, 1.0}, nbf, nbf, nbf, 1, 64, 64, one, false));
        ct2.push_back(job(Strided<false>{m.C, 1, nbf, 0, nbf}, Strided<false>{m.tmp, 1, nbf, 0, nbf},
                          EpiStore{m.tmp2, nbf, 0, 0, 1.0}, nbf, nbf, nbf, 1, 64, 64, one, false));
      }
    }
  }
  const size_t jbytes = job_bytes<JobTF>(nmol) * 2 + job_bytes<JobFF>(nmol) * 2 +
                        job_bytes<JobCas>(nmol) + job_bytes<JobTT>(nmol) * 3 +
                        job_bytes<JobW>(nmol) + job_bytes<JobK>(nmol) + job_bytes<JobTF>(nmol) * 2 +
                        job_bytes<JobTT>(nmol) + job_bytes<JobFF>(nmol) + 4096;
  char* jb = nullptr;
  CHECK(ws_get(c, W_BATCH_JOBS, jbytes, &jb));
  char* cursor = jb;
  Jobs J;
  J.n = nmol;
  CHECK(upload_jobs(c, mo1, bm(TU_MO1), bn(TU_MO1), cursor, &J.mo1, &J.mo1_wg));
  CHECK(upload_jobs(c, mo2, bm(TU_MO2), bn(TU_MO2), cursor, &J.mo2, &J.mo2_wg));
  CHECK(upload_jobs(c, cas, bm(TU_CASIDA), bn(TU_CASIDA), cursor, &J.cas, &J.cas_wg));
  CHECK(upload_jobs(c, rho, bm(TU_RHO), bn(TU_RHO), cursor, &J.rho, &J.rho_wg));
  CHECK(upload_jobs(c, wj, 128, 128, cursor, &J.w, &J.w_wg));
  CHECK(upload_jobs(c, sig, bm(TU_SIGMA), bn(TU_SIGMA), cursor, &J.sig, &J.sig_wg));
  CHECK(upload_jobs(c, hc1, 64, 64, cursor, &J.hc1, &J.hc1_wg));
  CHECK(upload_jobs(c, hc2, 64, 64, cursor, &J.hc2, &J.hc2_wg));
  CHECK(upload_jobs(c, exc, bm(TU_EXCHANGE), bn(TU_EXCHANGE), cursor, &J.exc, &J.exc_wg));
  CHECK(upload_jobs(c, rot, 64, 64, cursor, &J.rot, &J.rot_wg));
  CHECK(upload_jobs(c, cg3, 64, 64, cursor, &J.cg3, &J.cg3_wg));
  CHECK(upload_jobs(c, cg4, 64, 64, cursor, &J.cg4, &J.cg4_wg));
  CHECK(upload_jobs(c, ct1, 64, 64, cursor, &J.ct1, &J.ct1_wg));
  CHECK(upload_jobs(c, ct2, 64, 64, cursor, &J.ct2, &J.ct2_wg));
  J.nv = (int64_t)cg3.size();
  J.nmix = (int64_t)ct1.size();
  Mol* dm = nullptr;
  CHECK(ws_get(c, W_BATCH_MOLS, (size_t)nmol, &dm));
  HIP_TRY(c, hipMemcpyAsync(dm, P.mols.data(), nmol * sizeof(Mol), hipMemcpyHostToDevice, c->stream));
  P.dmols = dm;
  // host-side vectors above stay alive until here: wait for the copies
  HIP_TRY(c, hipStreamSynchronize(c->stream));

  // -------------------------------------------------------- iterations --
  std::vector<double> deps(nmol);
  std::vector<int> flag_h(nmol);
  std::vector<int64_t> first_ok(nmol, -1);
  std::vector<std::vector<double>> hist(nmol);
  const bool graph = (o->flags & QSGW_OPT_GRAPH) != 0;
  if (graph && c->stream == nullptr)
    return fail(c, QSGW_ERR_UNSUPPORTED, "graph capture needs a context on a non-default stream");
  Graphs gx;
  double ms_hot = 0.0, ms_eigM = 0.0, ms_eigF = 0.0;
  double ms_kernel[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t launches[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // kernel segments: A (MO transform, Casida build), B1 (rho, residues),
  // B2 (qsGW matrix, Fock build), C (rotation, update); the Casida eigensolve
  // follows A, the Fock eigensolve B2; the per-state diagonal outputs run
  // between B1 and B2 on the first iteration only
  auto seg = [&](int k, Spans* ks) -> int {
    if (k == 0)
      return x3 ? segment_a<float, Bf16x3>(c, P, J, ks)
                : fp32 ? segment_a<float, float>(c, P, J, ks) : segment_a<double, double>(c, P, J, ks);
    if (k == 1)
      return x3 ? segment_b<Bf16x3>(c, P, J, ks)
                : fp32 ? segment_b<float>(c, P, J, ks) : segment_b<double>(c, P, J, ks);
    if (k == 2) return segment_b2(c, P, J, ks);
    return segment_c(c, P, J, ks);
  };
  bool any_diag = false;
  for (int64_t i = 0; i < nmol; ++i) any_diag = any_diag || P.mols[i].diag != nullptr;
  const int seg_stage[4] = {kStageMo, kStageRes, kStageSigma, kStageFock};
  int status = QSGW_OK;
  for (int64_t it = 0; it < o->max_iter; ++it) {
    // stage spans: the kernel segments and the two eigensolves; kernel spans
    // inside the segments when they run eagerly
    Spans sp;
    sp.c = c;
    Spans* ks = graph ? nullptr : &sp;
    for (int k = 0; k < 4; ++k) {
      if (graph && !gx.x[k]) {
        // capture the segment once (nothing runs during capture), then replay
        hipGraph_t g = nullptr;
        HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const int rc = seg(k, nullptr);
        const hipError_t ec = hipStreamEndCapture(c->stream, &g);
        if (rc < 0) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        if (ec != hipSuccess) return fail(c, QSGW_ERR_HIP, "graph capture: %s", hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&gx.x[k], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
          gx.x[k] = nullptr;
          return fail(c, QSGW_ERR_HIP, "graph instantiate: %s", hipGetErrorString(ei));
        }
      }
      CHECK(sp.open(seg_stage[k]));
      if (graph) {
        HIP_TRY(c, hipGraphLaunch(gx.x[k], c->stream));
      } else {
        CHECK(seg(k, ks));
      }
      CHECK(sp.close());
      if (k == 1 && it == 0 && any_diag) {
        hipLaunchKernelGGL(kb_diag, dim3((unsigned)P.total[S_NBF]), dim3(256), 0, c->stream, P.dmols,
                           P.dpre[S_NBF], nmol);
        CHECK(launch_check(c, "kb_diag"));
      }
      if (k == 0 || k == 2) {
        CHECK(sp.open(k == 0 ? kStageEigRpa : kStageEigFock));
        CHECK(eig_buckets(c, k == 0 ? P.bM : P.bF));
        CHECK(sp.close());
      }
    }
    HIP_TRY(c, hipMemcpyAsync(deps.data(), P.deps, nmol * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(flag_h.data(), flags, nmol * sizeof(int), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (const auto& span : sp.v) {
      const double ms = elapsed(c, span.e0, span.e1);
      if (span.id >= kKernelBase) {
        ms_kernel[span.id - kKernelBase] += ms;
        launches[span.id - kKernelBase] += 1;
      } else if (span.id == kStageEigRpa) {
        ms_eigM += ms;
      } else if (span.id == kStageEigFock) {
        ms_eigF += ms;
      } else {
        ms_hot += ms;
      }
    }
    for (int64_t i = 0; i < nmol; ++i) {
      if (status >= 0) {
        if (flag_h[i] & 1)
          status = fail(c, QSGW_ERR_INVALID_ARG, "molecule %lld: orbital energies are not in aufbau order",
                        (long long)i);
        else if (flag_h[i] & 2)
          status = fail(c, QSGW_ERR_SOLVER, "molecule %lld: RPA instability (Omega^2 <= 0)", (long long)i);
        else if (!isfinite(deps[i]))
          status = fail(c, QSGW_ERR_NONFINITE, "molecule %lld: non-finite orbital energies", (long long)i);
      }
      hist[i].push_back(deps[i]);
      if (first_ok[i] < 0 && deps[i] < o->tol) first_ok[i] = it + 1;
      states[i].iteration++;
    }
    if (status < 0) break;
  }
  // solver info of the last call of each bucket
  for (auto* bs : {&P.bM, &P.bF})
    for (auto& b : *bs) {
      std::vector<int> info(b.mols.size());
      HIP_TRY(c, hipMemcpy(info.data(), b.info, info.size() * sizeof(int), hipMemcpyDeviceToHost));
      for (size_t j = 0; j < info.size(); ++j)
        if (info[j] != 0 && status >= 0)
          status = fail(c, QSGW_ERR_SOLVER, "molecule %lld: dsyevd info %d", (long long)b.mols[j], info[j]);
    }
  bool all = true;
  for (int64_t i = 0; i < nmol; ++i) {
    all = all && first_ok[i] > 0;
    if (reports) {
      const Mol& m = P.mols[i];
      const double b = (double)m.nbf, a = (double)m.naux, t = (double)m.ntr, oc = (double)m.nocc;
      qsgw_report& r = reports[i];
      memset(&r, 0, sizeof(r));
      r.iterations = (int64_t)hist[i].size();
      r.converged = first_ok[i] > 0;
      for (size_t k = 0; k < hist[i].size() && k < QSGW_REPORT_MAX_ITERS; ++k) r.max_deps[k] = hist[i][k];
      r.ms_stage[kStageMo] = ms_hot;
      r.ms_stage[kStageEigRpa] = ms_eigM;
      r.ms_stage[kStageEigFock] = ms_eigF;
      r.hot_flops = (3.0 * b + 1.0) * b * b * a + t * (t + 1.0) * a + 2.0 * a * t * t + b * (b + 1.0) * a * t +
                    2.0 * b * b * b * t + b * (b + 1.0) * a * oc + 2.0 * a * b * b + 6.0 * b * b * b;
      r.kernel_flops[kKMo1 - kKernelBase] = 2.0 * b * b * b * a;
      r.kernel_flops[kKMo2 - kKernelBase] = b * (b + 1.0) * b * a;  // symmetric output
      r.kernel_flops[kKCasida - kKernelBase] = t * (t + 1.0) * a;
      r.kernel_flops[kKRho - kKernelBase] = 2.0 * a * t * t;
      r.kernel_flops[kKW - kKernelBase] = b * (b + 1.0) * a * t;
      r.kernel_flops[kKSigma - kKernelBase] = 2.0 * b * b * b * t;
      r.kernel_flops[kKFock - kKernelBase] = b * (b + 1.0) * a * oc + 2.0 * a * b * b + 4.0 * b * b * b;
      for (int k = 0; k < 8; ++k) {
        r.ms_kernel[k] = ms_kernel[k];
        r.kernel_launches[k] = launches[k];
      }
    }
  }
  if (status < 0) return status;
  return all ? QSGW_OK : QSGW_NOT_CONVERGED;
}
