/*
 * libqsgw -- one RI quasiparticle self-consistent GW (qsGW) iteration on an
 * AMD Instinct MI355X (gfx950).
 *
 * The method is the one of "GPU acceleration of many-body perturbation theory
 * methods in MOLGW with OpenACC" (arXiv 2210.17093), section "Theoretical
 * background", with the two-electron integrals in resolution-of-identity
 * (RI) form (mu nu|lambda tau) = sum_P B^P_{mu nu} B^P_{lambda tau}:
 *
 *   LCAO, Eq. (3)            phi_m = sum_mu C_{mu m} phi_mu
 *   AO->MO, Eq. (16)         B^P_{mn} = sum_{mu nu} C_{mu m} B^P_{mu nu} C_{nu n}
 *   Casida, Eqs. (12)-(14)   closed-shell singlet, A = Delta + 2K, B = 2K,
 *                            K_{ia,jb} = sum_P B^P_{ia} B^P_{jb}, solved as
 *                            M = (A-B)^{1/2}(A+B)(A-B)^{1/2} = Delta^2 + 4 sqrt(Delta) K sqrt(Delta)
 *   residues, Eq. (18)       w^s_{mn} = sqrt(2) sum_P B^P_{mn} sum_{ia} B^P_{ia} (X+Y)^s_{ia}
 *   self-energy, Eq. (17)    Sigma_{mn}(omega) = sum_{i s} w^s_{mi} w^s_{ni} / (omega - eps_i + Omega_s - i eta)
 *                                              + sum_{a s} w^s_{ma} w^s_{na} / (omega - eps_a - Omega_s + i eta)
 *   qsGW potential, Eq. (19) V_{mn} = 1/2 Re[Sigma_{mn}(eps_m) + Sigma_{mn}(eps_n)]
 *   Hamiltonian, Eq. (6)     F = h + J - K + C V C^T, with J, K of Eqs. (7), (9), (10)
 *   eigenproblem, Eq. (4)    F C' = C' eps' (S = I: orthonormal synthetic AO basis)
 *
 * Conventions shared by every entry point:
 *   - Every array argument is a DEVICE pointer, FP64, row-major, contiguous,
 *     allocated and owned by the caller.  The library never frees a caller
 *     pointer and keeps none past the call.
 *   - Sizes are int64_t; element offsets are computed in 64-bit.
 *   - n_occ occupied orbitals are the lowest ones (aufbau); n_v = nbf - nocc;
 *     transitions are t = i * n_v + (a - nocc) for 0 <= i < nocc <= a < nbf;
 *     ntr = nocc * n_v.
 *   - Work is queued on the context's HIP stream and is asynchronous unless
 *     stated otherwise.  The context owns its workspace (grown on demand with
 *     hipMalloc, released by qsgw_ctx_destroy).
 *   - Return value: QSGW_OK, QSGW_NOT_CONVERGED (results valid), or a
 *     negative error; qsgw_last_error() returns a message for the context.
 *   - Every entry point that reads floating-point input arrays checks them
 *     for NaN and infinity on the device (one pass over each input, then one
 *     read-back, so the call synchronizes its stream once before its work
 *     is queued) and returns QSGW_ERR_NONFINITE naming the array; nothing
 *     else runs then.
 *   - One context per host thread.  Calls on one context must not overlap.
 */
#ifndef QSGW_H
#define QSGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSGW_VERSION 1

/* Status codes. */
#define QSGW_OK 0
#define QSGW_NOT_CONVERGED 1
#define QSGW_ERR_INVALID_ARG (-1)
#define QSGW_ERR_NONFINITE (-2)
#define QSGW_ERR_HIP (-3)
#define QSGW_ERR_SOLVER (-4)
#define QSGW_ERR_ALLOC (-5)
#define QSGW_ERR_UNSUPPORTED (-6)

/* Arithmetic of the contractions (MO transform, RPA build, residues). */
#define QSGW_PREC_FP64 0
#define QSGW_PREC_FP32 1       /* FP32 matrix-core products, FP64 accumulation across K chunks */
/* Split-BF16 products: every FP32 operand x is split into x = hi + lo (hi =
   bf16(x), lo = bf16(x - hi)) and a*b is taken as hi*hi + hi*lo + lo*hi on
   BF16 matrix cores with FP32 accumulation (relative error about 2^-16 per
   product term), FP64 across K chunks.  It applies to the Casida build, the
   residue products and the far-from-pole part of the qsGW matrix; the MO
   transform runs on the FP32 matrix cores.  In qsgw_iterate_batched it
   covers the Casida, rho' and residue products (the qsGW product stays FP64
   there). */
#define QSGW_PREC_SPLIT_BF16 2

/* qsgw_sigma modes. */
#define QSGW_SIGMA_QS_MATRIX 0
#define QSGW_SIGMA_DIAG_GRID 1
#define QSGW_SIGMA_DIAG_SELF 2

/* Fock update modes of qsgw_iterate, Eq. (6). */
#define QSGW_FOCK_FULL_JK 0 /* F = h + J[D] - K[D] + Vc, D from the current orbitals */
/* F = h + Vc: the mean field is frozen.  h is then the whole frozen mean-field
 * Hamiltonian F0 = T + V_ext + J[D0] - K[D0] of a reference density D0 (for
 * example the Hartree-Fock Fock matrix of the start); J and K are not rebuilt.
 * From a start whose density is D0 the first iteration equals that of
 * QSGW_FOCK_FULL_JK with the matching one-body h. */
#define QSGW_FOCK_FROZEN 1

#define QSGW_REPORT_MAX_ITERS 64

typedef struct qsgw_ctx qsgw_ctx;

/* Create a context bound to a HIP stream (hipStream_t passed as void*; NULL
 * means the null stream of the current device).  The context also creates a
 * rocBLAS handle on that stream for the dense eigensolver. */
int qsgw_ctx_create(qsgw_ctx** ctx, void* hip_stream);
int qsgw_ctx_destroy(qsgw_ctx* ctx);
/* Last error message of this context ("" if none).  Owned by the context. */
const char* qsgw_last_error(const qsgw_ctx* ctx);
/* Returns QSGW_VERSION. */
int qsgw_version(void);
/* Host timing of the last call's stages, milliseconds (HIP events on the
 * context stream); fills up to n entries in the order
 * {mo_transform, rpa_build, eig_rpa, residues, sigma, fock, eig_fock}. */
int qsgw_last_stage_ms(const qsgw_ctx* ctx, double* ms, int n);

/*
 * AO->MO transform of the RI tensor, Eq. (16):
 *   B_mo[P][m][n] = sum_{mu,nu} C[mu][m] B_ao[P][mu][nu] C[nu][n].
 * B_ao: [naux][nbf][nbf], symmetric in its last two indices.
 * C:    [nbf][nbf], column m holds MO m.
 * B_mo: [naux][nbf][nbf] out; written exactly symmetric in (m, n).
 * precision: any QSGW_PREC_*; QSGW_PREC_SPLIT_BF16 runs FP32 products here.
 * Errors: nbf < 1, naux < 1, NULL pointers, an unknown precision.
 */
int qsgw_mo_transform(qsgw_ctx* ctx, int64_t nbf, int64_t naux, const double* B_ao,
                      const double* C, double* B_mo, int precision);

/*
 * Hermitian Casida matrix, Eqs. (12)-(14), closed-shell singlet:
 *   sqrt_delta[t] = sqrt(eps[a] - eps[i]),
 *   M[t][u] = delta_tu Delta_t^2 + 4 sqrt_delta[t] (sum_P B_mo[P][i][a] B_mo[P][j][b]) sqrt_delta[u]
 * for t = (i, a), u = (j, b).  M is [ntr][ntr], written exactly symmetric.
 * B_mo: [naux][nbf][nbf]; eps: [nbf] ascending (eps[a] > eps[i] required).
 * precision: any QSGW_PREC_*; sqrt_delta and the diagonal stay FP64.
 * Errors: 0 < nocc < nbf violated; an unknown precision.
 */
int qsgw_rpa_build(qsgw_ctx* ctx, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                   const double* eps, double* M, double* sqrt_delta, int precision);

/* Solvers of the Casida eigenproblem M Z = Z Omega^2 (Eq. (12)), chosen per
 * context with qsgw_set_eigensolver.  They apply to qsgw_rpa_solve and to the
 * Casida eigensolves inside qsgw_iterate and qsgw_gw_unrestricted (the Fock
 * eigensolves and the batched path always use rocSOLVER dsyevd). */
#define QSGW_EIG_AUTO 0      /* the two-stage solver for n >= 8192, dsyevd below (default) */
#define QSGW_EIG_ROCSOLVER 1 /* rocSOLVER dsyevd (one-stage tridiagonal reduction) */
/* Two-stage reduction, all FP64: dense -> band of half-width 64 by blocked
 * Householder panels whose two-sided updates are matrix products, band ->
 * tridiagonal by bulge chasing, rocSOLVER divide and conquer (dstedc) on the
 * tridiagonal matrix, then both back-transformations (the bulge-chasing
 * reflectors in blocks of 64 sweeps, the panel reflectors as block
 * reflectors).  Inside qsgw_iterate and qsgw_gw_unrestricted (and so the
 * open-shell iteration) only the projection of the auxiliary basis on the
 * eigenvectors is needed: the back-transformations act on its
 * N_aux columns and the tridiagonal eigenproblem is solved by divide and
 * conquer whose merges act on those columns too (blocks up to the tile
 * table's dc_leaf by dstedc), so no eigenvector matrix is formed.  Below
 * n = 256 it calls dsyevd. */
#define QSGW_EIG_TWO_STAGE 2

/* Selects the Casida eigensolver of the context (QSGW_EIG_*).  Eigenvectors
 * of equal quality either way; signs, and rotations inside degenerate
 * eigenspaces, may differ between solvers.
 * Errors: an unknown solver. */
int qsgw_set_eigensolver(qsgw_ctx* ctx, int solver);

/*
 * Dense symmetric eigensolve of the Casida matrix (the context's solver,
 * qsgw_set_eigensolver), kept apart from the hot path: M Z = Z Omega^2.
 * M_to_Z: [ntr][ntr] in; on return holds Z column-major, i.e. row s of the
 *         row-major view is the eigenvector of Omega[s].
 * Omega:  [ntr] out, ascending, Omega_s = sqrt of the eigenvalue.
 * Errors: QSGW_ERR_SOLVER if the solver fails or an eigenvalue is <= 0 (RPA
 * instability).  Synchronizes the context stream.
 */
int qsgw_rpa_solve(qsgw_ctx* ctx, int64_t ntr, double* M_to_Z, double* Omega);

/*
 * Screened-interaction residues, Eq. (18), for excitations
 * s in [s_begin, s_begin + s_count):
 *   (X+Y)[t][s] = sqrt_delta[t] Z[s][t] / sqrt(Omega[s])
 *   rho[P][s]   = sum_t B_mo[P][i_t][a_t] (X+Y)[t][s]
 *   w[m][n][s - s_begin] = sqrt(2) sum_P B_mo[P][m][n] rho[P][s]
 * Z: [ntr][ntr] as returned by qsgw_rpa_solve; Omega: [ntr].
 * w: [nbf][nbf][s_count] out, written exactly symmetric in (m, n).
 * wh: NULL, or [nbf][nbf][s_count] out: the pole-weighted copy used by the
 *   qsGW matrix of qsgw_sigma,
 *   wh[m][n][s] = w[m][n][s] Re 1/(eps_m - eps_n +- (Omega_s - i eta))
 *   ("+" for occupied n, "-" for empty n); then eps ([nbf]) and eta > 0 are
 *   required, otherwise they are ignored.
 * precision: any QSGW_PREC_* (reduced precisions round B_mo, Bt, Z and rho
 *   to FP32 before their products; w and wh are still written in FP64).
 * Errors: s range outside [0, ntr); an unknown precision; wh without
 * eps or with eta <= 0.
 */
int qsgw_residues(qsgw_ctx* ctx, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                  const double* sqrt_delta, const double* Z, const double* Omega,
                  int64_t s_begin, int64_t s_count, double* w, double* wh, const double* eps,
                  double eta, int precision);

/*
 * GW self-energy from residues of ns excitations, Eq. (17).
 * w:     [nbf][nbf][ns] as written by qsgw_residues;
 * wh:    NULL, or the pole-weighted copy written by qsgw_residues with the
 *        same eps, Omega and eta (QS_MATRIX mode only; saves recomputing the
 *        weights); ignored by DIAG_GRID;
 * Omega: [ns], the excitation energies of those ns columns.
 * mode QSGW_SIGMA_QS_MATRIX, Eq. (19):
 *   out[m][n] (+)= 1/2 (G[m][n] + G[n][m]),
 *   G[m][n] = sum_{k,s} w[m][k][s] w[n][k][s] Re 1/(eps_m - eps_k +- (Omega_s - i eta))
 *   ("+" for occupied k, "-" for empty k).  omega, nomega, states, nstates unused.
 * mode QSGW_SIGMA_DIAG_GRID, Eq. (17) with m = n:
 *   out[j][l] (+)= Sigma_{mm}(omega[l]), m = states[j], complex128 stored as
 *   interleaved (re, im) pairs: out is [nstates][nomega][2].
 *   omega: [nomega] device; states: [nstates] device int64.
 * mode QSGW_SIGMA_DIAG_SELF, Eq. (17) with m = n at each state's own energy:
 *   out[j][0..2] (+)= Re Sigma_mm(eps_m), Im Sigma_mm(eps_m) and
 *   Re dSigma_mm/domega at omega = eps_m, m = states[j]; out is [nstates][3].
 *   states: [nstates] device int64; omega, nomega unused.
 * accumulate = 1 adds into out (for streamed excitation blocks), 0 overwrites.
 * Errors: eta <= 0; states out of range (checked on the host only for nstates
 * <= 0; device indexes are clamped-checked and flagged as INVALID_ARG).
 */
int qsgw_sigma(qsgw_ctx* ctx, int mode, int64_t nbf, int64_t nocc, int64_t ns, const double* w,
               const double* wh, const double* eps, const double* Omega, double eta,
               const double* omega, int64_t nomega, const int64_t* states, int64_t nstates,
               double* out, int accumulate);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * QSGW_SIGMA_QS_MATRIX mode of qsgw_sigma (same arguments, same result up to
 * the rounding order of its K-split) without any allocation.  Its split-K
 * partial sums and its finite-input flag live in one static device array of
 * 64 MiB that the library holds on every device it runs on until the process
 * ends; the K-split is capped at what it holds (at most 64 slices), so nbf is
 * limited to 2896 (QSGW_ERR_INVALID_ARG above).  The call still synchronizes
 * once to read the finite-input flag, and records no stage times.  All calls
 * on one device share that array: calls that overlap on one device (two
 * contexts or streams at once) race and must be serialized by the caller.
 */
int qsgw_sigma_qs_noalloc(qsgw_ctx* ctx, int64_t nbf, int64_t nocc, int64_t ns, const double* w,
                          const double* wh, const double* eps, const double* Omega, double eta,
                          double* out, int accumulate);

/*
 * qsMP2 potential: the correlation part of the MP2 self-energy, Eq. (20),
 * made Hermitian as in Eq. (21); closed shell, real orbitals:
 *   V[m][n] (+)= 1/2 Re[Sigma_mn(eps_n) + Sigma_nm(eps_m)],
 *   Sigma_mn(w) = sum_{p, i, a} (mp|ia) [2 (pn|ai) - X_pian] g_pia(w),
 *   X = (pi|an) for empty p, (pa|in) for occupied p,
 *   g = 1 / (w + eps_a - eps_i - eps_p - i eta) for occupied p,
 *       1 / (w + eps_i - eps_a - eps_p + i eta) for empty p,
 * i occupied, a empty, p any state, (kl|rs) = sum_P B_mo[P][k][l] B_mo[P][r][s].
 * The second-order exchange term for occupied p pairs the indices as (pa|in),
 * the form the antisymmetrised spin-orbital second-order self-energy gives.
 * B_mo: [naux][nbf][nbf] device, symmetric in (k, l) (as qsgw_mo_transform
 *       writes it); eps: [nbf] device; V: [nbf][nbf] device out, written
 *       exactly symmetric.
 * occ_block: occupied states i per block of transitions (i, a); 0 picks the
 *       largest block whose two [nbf][nbf][block transitions] FP64 work
 *       arrays fit in 16 GiB.  More than one block also keeps (ni|pa) for
 *       every occupied i ([nocc][nbf][ntr] FP64).  The workspace is owned by
 *       the context and kept for later calls.
 * accumulate = 1 adds into V, 0 overwrites.
 * precision: QSGW_PREC_FP64 only (others return QSGW_ERR_UNSUPPORTED).
 * Errors: 0 < nocc < nbf violated, naux < 1, eta <= 0 or not finite, NULL
 * pointers, occ_block < 0, nbf * (transitions of a block) >= 2^32,
 * QSGW_ERR_ALLOC when the workspace cannot be allocated.  Asynchronous on the
 * context stream; the time of the call is reported as the sigma stage of
 * qsgw_last_stage_ms.
 */
int qsgw_mp2_sigma(qsgw_ctx* ctx, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                   const double* eps, double eta, double* V, int64_t occ_block, int accumulate,
                   int precision);

/*
 * Four-index AO->MO transform, Eq. (16), on explicit integrals (the route
 * without the RI factorisation), for a slab of the first MO index:
 *   eri_mo[m - m_begin][n][k][l] = sum_{mu nu lambda tau} C[mu][m] C[nu][n] C[lambda][k]
 *                                  C[tau][l] eri_ao[mu][nu][lambda][tau],
 *   m in [m_begin, m_begin + m_count), n, k, l in [0, nbf).
 * Four quarter transforms, one GEMM each (8 m_count nbf^4 FLOPs); a smaller
 * slab lowers the memory of the intermediates and the arithmetic intensity
 * of the first quarter (it reads the whole AO tensor once per call).
 * eri_ao: [nbf][nbf][nbf][nbf] device; C: [nbf][nbf] device, column m = MO m;
 * eri_mo: [m_count][nbf][nbf][nbf] device out, also used as scratch for the
 *   second quarter (must not overlap eri_ao or C).  The context keeps one
 *   [m_count][nbf][nbf][nbf] FP64 workspace.
 * precision: QSGW_PREC_FP64 only (others return QSGW_ERR_UNSUPPORTED).
 * Errors: nbf < 1, NULL pointers, a slab outside [0, nbf), QSGW_ERR_UNSUPPORTED
 * when nbf^3 strides exceed the tile loader's 32-bit offsets (nbf above about
 * 560), QSGW_ERR_ALLOC.  Asynchronous; timed as the MO stage of
 * qsgw_last_stage_ms.
 */
int qsgw_ao2mo_4center(qsgw_ctx* ctx, int64_t nbf, const double* eri_ao, const double* C,
                       int64_t m_begin, int64_t m_count, double* eri_mo, int precision);

/*
 * Open-shell (spin-unrestricted) GW potential, Eqs. (12)-(19) with the spin
 * labels sigma, sigma' kept: each spin has its own MO tensor, energies and
 * occupation.  Transitions t = (i, a, sigma) of both spins (alpha first, each
 * i-major) share one direct-RPA Casida problem,
 *   M = Delta^2 + 2 sqrt(Delta) K sqrt(Delta),  K[t][u] = sum_P B^{sigma P}_{ia} B^{sigma' P}_{jb},
 * solved inside the call by the context's Casida eigensolver
 * (qsgw_set_eigensolver); then for each spin sigma
 *   w[m][n][s] = sum_P B^{sigma P}_{mn} rho_{P s},  rho = sum_t B_t sqrt(Delta_t) Z[s][t] / sqrt(Omega_s),
 *   V_sigma[m][n] = 1/2 (G[m][n] + G[n][m]),
 *   G[m][n] = sum_{k,s} w[m][k][s] w[n][k][s] Re 1/(eps_m - eps_k +- (Omega_s - i eta))
 * with eps, the occupied range and "+" for k < nocc of that spin.
 * B_mo_a, B_mo_b: [naux][nbf][nbf] device (each spin's MO tensor, as
 *   qsgw_mo_transform writes it); eps_a, eps_b: [nbf] device, ascending.
 * V_a, V_b: [nbf][nbf] device out, written exactly symmetric.
 * Omega_out: NULL, or [nocc_a (nbf - nocc_a) + nocc_b (nbf - nocc_b)] device
 *   out, the excitation energies ascending.
 * precision: QSGW_PREC_FP64 only (others return QSGW_ERR_UNSUPPORTED).
 * Errors: 0 < nocc_a, nocc_b < nbf violated, naux < 1, eta <= 0, NULL
 * pointers, more than 46340 transitions, an empty transition energy
 * (INVALID_ARG), QSGW_ERR_SOLVER on an RPA instability.  Synchronizes the
 * context stream; qsgw_last_stage_ms then reports the rpa_build (transitions,
 * gather, Casida product), eig_rpa, residues and sigma stages of the call.
 */
int qsgw_gw_unrestricted(qsgw_ctx* ctx, int64_t nbf, int64_t naux, int64_t nocc_a, int64_t nocc_b,
                         const double* B_mo_a, const double* B_mo_b, const double* eps_a,
                         const double* eps_b, double eta, double* V_a, double* V_b,
                         double* Omega_out, int precision);

/*
 * Open-shell Fock update of both spins, Eqs. (4), (6), (7), (9), (10) with
 * explicit spins, in the MO basis of each spin's current orbitals C_sigma:
 *   F_sigma = C_sigma^T h C_sigma + J - K_sigma + V_sigma,
 *   J[m][n] = sum_P B^{sigma P}_mn (t^alpha_P + t^beta_P),  t^s_P = sum_{i < nocc_s} B^{s P}_ii,
 *   K_sigma[m][n] = sum_P sum_{i < nocc_sigma} B^{sigma P}_mi B^{sigma P}_ni,
 * then F_sigma = U diag(eps') U^T and C_sigma <- C_sigma U, each column's
 * largest-magnitude entry made positive.
 * B_mo_a, B_mo_b: [naux][nbf][nbf] device, the MO tensors of the current C_a, C_b;
 * h: [nbf][nbf] device (AO basis, orthonormal); V_a, V_b: [nbf][nbf] device, the
 *   spins' correlation potentials in their current MO bases (qsgw_gw_unrestricted);
 * eps_a, eps_b: [nbf] device out; C_a, C_b: [nbf][nbf] device in/out.
 * Errors: 0 < nocc_a, nocc_b < nbf violated, naux < 1, NULL pointers,
 * QSGW_ERR_SOLVER if dsyevd fails.  Synchronizes the context stream; timed as
 * the fock stage of qsgw_last_stage_ms.
 */
int qsgw_fock_unrestricted(qsgw_ctx* ctx, int64_t nbf, int64_t naux, int64_t nocc_a, int64_t nocc_b,
                           const double* B_mo_a, const double* B_mo_b, const double* h,
                           const double* V_a, const double* V_b, double* eps_a, double* eps_b,
                           double* C_a, double* C_b);

/*
 * One-body matrix that makes (eps0, C0) a Hartree-Fock fixed point of
 * Eq. (6) with Sigma_c = 0:  h = C0 diag(eps0) C0^T - J[D0] + K[D0],
 * D0 = C0[:, :nocc] C0[:, :nocc]^T (Eq. (9)), J and K from Eqs. (7), (10).
 * h: [nbf][nbf] out.  Used to build synthetic problems.
 */
int qsgw_hf_core(qsgw_ctx* ctx, int64_t nbf, int64_t naux, int64_t nocc, const double* B_ao,
                 const double* C0, const double* eps0, double* h);

/* Problem, state, options and report of qsgw_iterate. */
typedef struct {
  int64_t nbf;
  int64_t naux;
  int64_t nocc;
  const double* B_ao; /* device [naux][nbf][nbf], symmetric in (mu, nu) */
  const double* h;    /* device [nbf][nbf], one-body part T + V_ext of Eq. (6) */
} qsgw_problem;

typedef struct {
  double* eps;       /* device [nbf], in/out: orbital energies, ascending */
  double* C;         /* device [nbf][nbf], in/out: MO coefficients, orthonormal columns */
  double* Vc;        /* device [nbf][nbf] or NULL, out: last AO-basis potential C V C^T;
                        read back as the previous potential when mix != 1 and iteration > 0 */
  int64_t iteration; /* in/out: iterations done so far (0 at the start) */
  double* diag;      /* device [nbf][4] or NULL, out: for the first iteration of the call, per
                        state m at the iteration's input energies, Eq. (17) with m = n:
                        Re Sigma_mm(eps_m), Im Sigma_mm(eps_m), Re dSigma_mm/domega(eps_m),
                        and the exchange diagonal Sigma_x,mm = -sum_{i occ, P} (B^P_mi)^2 */
} qsgw_state;

typedef struct {
  int precision;    /* QSGW_PREC_* */
  double eta;       /* > 0, Ha */
  double tol;       /* converged when max_m |eps'_m - eps_m| < tol */
  int64_t max_iter; /* iterations in this call, >= 1 */
  double mix;       /* Vc <- mix Vc + (1 - mix) Vc_prev, in (0, 1]; 1 = no mixing */
  int fock_mode;    /* QSGW_FOCK_FULL_JK */
  int64_t s_block;  /* excitations per streamed residue block; 0 = automatic */
  int64_t flags;    /* QSGW_OPT_* bits */
  double near_pole; /* reduced precisions, qsgw_iterate: terms of the qsGW product (Eq. 19)
                       with |eps_m - eps_k +- Omega_s| below this (Ha) are summed in FP64, the
                       rest on FP32 (or split-BF16) matrix cores; 0 = 0.05 Ha */
  const float* warm_start; /* qsgw_iterate only: NULL, or device [nbf] FP32 predicted shifts
                       delta_m (the learned warm start); the call first replaces the state's
                       (eps, C) by the warm start of qsgw_warm_start built from them, then
                       iterates.  qsgw_iterate_batched requires NULL. */
  int64_t diis;     /* qsgw_iterate only: 0 = off, or m in [2, 16]: Pulay's DIIS on the Fock
                       matrix of Eq. (6) (direct inversion in the iterative subspace; Pulay,
                       Chem. Phys. Lett. 73, 393 (1980) and J. Comput. Chem. 3, 556 (1982)),
                       an accelerator of the fixed point the paper leaves open: each
                       iteration's Fock matrix F (AO basis, S = I) is kept with its error
                       e = F D - D F (D of Eq. (9) from the orbitals that built F) among the
                       last m pairs, and the matrix diagonalised is sum_i c_i F_i with the c
                       minimising ||sum_i c_i e_i|| subject to sum_i c_i = 1 (the first
                       iteration of a history is the plain step; a singular system takes the
                       newest F).  The history lives in the context and continues across
                       calls; a state with iteration 0, another N_b or another m starts a new
                       one, so interleaved molecules need one context each.  Needs mix 1
                       (QSGW_ERR_INVALID_ARG otherwise). */
} qsgw_options;

/* qsgw_options.flags, qsgw_iterate_batched only: run the kernel segments
 * between eigensolves from hipGraphs captured on the first iteration. */
#define QSGW_OPT_GRAPH 1
/* qsgw_options.flags, qsgw_iterate with a reduced precision only: after the
 * reduced-precision iterations stop (converged or max_iter), run one more
 * iteration in FP64 from where they stopped (refinement pass).  The report
 * counts it: its last max_deps entry is the FP64 iteration's, and converged
 * and the return code are that iteration's. */
#define QSGW_OPT_REFINE 2
/* qsgw_options.flags, qsgw_iterate only: each iteration's correlation
 * potential is the qsMP2 potential of Eqs. (20)-(21) (as qsgw_mp2_sigma,
 * automatic blocks) instead of the qsGW one; the Casida problem is not built.
 * Needs precision QSGW_PREC_FP64 and state.diag NULL (QSGW_ERR_UNSUPPORTED
 * otherwise); its time is reported as the sigma stage. */
#define QSGW_OPT_QSMP2 4
/* qsgw_options.flags, qsgw_iterate only, for timing the hot path apart from
 * the Casida eigensolve: each iteration still builds its Casida matrix (into
 * a separate buffer) but, instead of solving it, takes the eigenpairs the
 * context kept from its last solved Casida matrix.  The library checks that
 * the new matrix is bitwise the solved one (an order-independent fingerprint
 * of its bit patterns) and returns QSGW_ERR_INVALID_ARG otherwise, so the
 * results are those of a full iteration.  The eig_rpa stage then reports
 * 0 ms.  Not combinable with QSGW_OPT_QSMP2. */
#define QSGW_OPT_REPLAY_EIG 8

typedef struct {
  int64_t iterations; /* iterations done in this call */
  int converged;      /* 1 if the last iteration met tol */
  double max_deps[QSGW_REPORT_MAX_ITERS]; /* max |d eps| of each iteration of this call */
  double ms_stage[7];      /* summed over the call: mo_transform, rpa_build, eig_rpa,
                              residues, sigma, fock, eig_fock */
  double hot_flops;        /* algorithmic FLOPs of one iteration's hot path */
  double ms_kernel[8];     /* summed over the call, per kernel: AO->MO half 1, AO->MO half 2,
                              Casida gather+product, residue rho, residue w, qsGW matrix
                              product, qsGW reduce, Fock build */
  double kernel_flops[8];  /* algorithmic FLOPs of one iteration, same kernel order */
  int64_t kernel_launches[8]; /* launches of each kernel in the call */
} qsgw_report;

/*
 * qsGW iterations, all on the device: per iteration Eq. (16) -> Casida
 * (eigensolve apart) -> Eq. (18) -> Eqs. (17), (19) -> Eq. (6) in the basis
 * of the current orbitals -> eigensolve of Eq. (4) -> C' = C U.
 * Updates st->eps, st->C (and st->Vc) in place; stops after max_iter or when
 * converged.  Synchronizes once per iteration to read max|d eps|.
 * Returns QSGW_OK if converged, QSGW_NOT_CONVERGED otherwise.
 */
int qsgw_iterate(qsgw_ctx* ctx, const qsgw_problem* prob, qsgw_state* st, const qsgw_options* opt,
                 qsgw_report* rep);

/*
 * Open-shell (spin-unrestricted) qsGW iterations, Eqs. (4), (6), (12)-(19)
 * with explicit spins, all on the device: per iteration the MO transform of
 * each spin's orbitals (Eq. 16), the open-shell GW potential of both spins
 * from one Casida problem over the transitions of both spins
 * (qsgw_gw_unrestricted), and the open-shell Fock update with its
 * eigensolve (qsgw_fock_unrestricted).  Converged when the largest change
 * of any orbital energy of either spin, max_m |eps'_m - eps_m|, is below
 * opt->tol.
 * prob: nbf, naux, B_ao, h as in qsgw_iterate, with prob->nocc the number of
 *   alpha electrons; nocc_b: the number of beta electrons.
 * st_a, st_b: each spin's eps and C (in/out) and iteration count (advanced);
 *   Vc and diag must be NULL.
 * opt: eta, tol, max_iter are used; precision must be QSGW_PREC_FP64, mix 1,
 *   fock_mode QSGW_FOCK_FULL_JK, flags 0, s_block 0, warm_start NULL
 *   (QSGW_ERR_UNSUPPORTED otherwise).
 * rep: NULL or the report (iterations, converged, max_deps per iteration,
 *   ms_stage summed over the call, hot_flops of one iteration; the per-kernel
 *   fields are zero).
 * Returns QSGW_OK if converged, QSGW_NOT_CONVERGED otherwise, or an error of
 * the entry points it calls.  Synchronizes several times per iteration.
 */
int qsgw_iterate_unrestricted(qsgw_ctx* ctx, const qsgw_problem* prob, int64_t nocc_b,
                              qsgw_state* st_a, qsgw_state* st_b, const qsgw_options* opt,
                              qsgw_report* rep);

/*
 * Batched qsGW iterations for nmol independent molecules of different sizes
 * (hundreds of small molecules per call).
 * probs, states: host arrays of nmol entries whose pointers are device
 * pointers as in qsgw_iterate; reports: host array of nmol entries or NULL.
 * The arrays are read during the call only.
 * Every stage runs as one launch over all molecules: grouped matrix-core
 * GEMMs (a job table with one entry per molecule, each workgroup finding its
 * molecule by binary search) and segment kernels for the element-wise steps.
 * Each molecule's arithmetic is that of qsgw_iterate (same tile shapes, K
 * splits and epilogues).  The Casida and Fock eigensolves are rocSOLVER
 * strided-batched dsyevd calls, one per size bucket: each matrix is stored
 * padded to its bucket size with zero coupling and a diagonal above its
 * Gershgorin bound, so its own eigenpairs come first.  With QSGW_OPT_GRAPH
 * the kernel segments between eigensolves are captured into hipGraphs on the
 * first iteration and replayed on every iteration (this needs a context
 * created on a stream other than the legacy default stream).
 * Every molecule runs opt->max_iter iterations (opt->s_block must be 0;
 * precision FP64, FP32 (MO transform, Casida, rho' and residue products on
 * the FP32 matrix cores) or SPLIT_BF16 (Casida, rho' and residue products as
 * split-BF16 products, the MO transform on the FP32 matrix cores); the qsGW
 * product and the Fock update stay FP64; with opt->mix != 1 every state needs a Vc buffer,
 * mixed as in qsgw_iterate from the molecule's own iteration count; the
 * diag outputs of a state are written during the call's first iteration);
 * a report's converged field says
 * whether some iteration met tol, max_deps holds every iteration's
 * max |d eps|.  Times are whole-batch figures, the same in every report:
 * ms_stage[2] and ms_stage[6] the Casida and Fock eigensolves, ms_stage[0]
 * every other step; ms_kernel and kernel_launches per kernel group when the
 * segments run eagerly (zero with QSGW_OPT_GRAPH).  hot_flops and
 * kernel_flops are the molecule's own algorithmic FLOPs per iteration.
 * Synchronizes once per iteration.
 * Returns QSGW_OK if every molecule met tol, QSGW_NOT_CONVERGED otherwise;
 * an error names the first failing molecule.
 */
int qsgw_iterate_batched(qsgw_ctx* ctx, int64_t nmol, const qsgw_problem* probs,
                         qsgw_state* states, const qsgw_options* opt, qsgw_report* reports);

/*
 * Tile table of the context (written by the autotuner, tune.py).  spec is a
 * comma-separated list of key=value: mo1, rho, sigma take 64x64, 128x64 or
 * 128x128; mo2, casida, exchange (symmetric products) 64x64 or 128x128;
 * sigma_target, rho_target, exchange_target, mp2_target (integers in
 * [64, 2^20]) are the workgroup counts a K-split aims for when a product has
 * few output tiles (mp2_target: the contraction of qsgw_mp2_sigma, whose
 * tile shape is sigma's);
 * persistent (integer in [0, 8]): for the grouped products of
 * qsgw_iterate_batched, 0 launches one workgroup per tile, n > 0 a
 * persistent grid of n workgroups per compute unit that walk contiguous
 * tile ranges; dc_leaf (integer in [16, 46340]): the two-stage solver's
 * projection (inside qsgw_iterate) solves the tridiagonal eigenproblem by
 * divide and conquer, halving blocks larger than dc_leaf and handing blocks
 * up to that order to rocSOLVER dstedc; panel_coop (0 or 1): 1 factors each
 * Householder panel of the two-stage solver's dense -> band stage in one
 * cooperative launch (the panel's rows held on chip, grid barriers between
 * columns; where the device cannot hold every workgroup at once it falls back
 * by itself), 0 in one launch per column.  Keys not given keep their
 * defaults (mo1=128x64, mo2=64x64, casida=128x128, rho=128x128,
 * sigma=64x64, exchange=64x64, 4096, 2048, 2048, mp2_target=32768,
 * persistent=0, dc_leaf=6144, panel_coop=1); NULL or "" restores all
 * defaults.  Every later product and
 * iteration on the context uses the table (results change only by rounding
 * order).  qsgw_get_tiles writes the current table in the same format.
 */
int qsgw_set_tiles(qsgw_ctx* ctx, const char* spec);
int qsgw_get_tiles(qsgw_ctx* ctx, char* buf, int64_t size);

/* ------------------------------------------------------------------------
 * Learned warm start.  A network 16 -> 128 -> 128 -> 1 with GELU
 * activations maps per-state features of a molecule's first iteration to the
 * state's converged qsGW shift delta_m = eps_m(converged) - eps_m(start); the
 * iteration then starts from eps0 + delta and the unchanged orbitals.
 * Parameters are one FP32 array of QSGW_MLP_NPARAMS values laid out as
 * W1[128][16], b1[128], W2[128][128], b2[128], w3[128], b3[1]
 * (z = W x + b per layer, y = w3 . a2 + b3).  All arrays are device pointers.
 * ------------------------------------------------------------------------ */
#define QSGW_MLP_NPARAMS 18817
#define QSGW_MLP_NFEAT 16

/*
 * Features of every state m of one molecule, from its orbital energies eps
 * ([nbf], the first iteration's input) and the diag output of that
 * iteration ([nbf][4], see qsgw_state.diag):
 *   0 eps_m, 1 Sigma_x,mm, 2 Re Sigma_mm(eps_m), 3 Re dSigma_mm/domega,
 *   4 nocc/nbf, 5 eps_LUMO - eps_HOMO, 6 Im Sigma_mm(eps_m),
 *   7 Z = 1/(1 - dSigma/domega), 8 occupied (1/0), 9 eps_m - eps_HOMO,
 *   10 eps_m - eps_LUMO, 11 nbf/120, 12 m/nbf, 13 Z Re Sigma_mm(eps_m)
 *   (the linearized shift at a Hartree-Fock start), 14 |dSigma/domega| > 1
 *   (1/0), 15 constant 1.
 * X: [nbf][16] FP32 out, (f - mean[q]) / scale[q] when mean and scale
 * ([16] FP32) are given, raw values when both are NULL.
 */
int qsgw_mlp_features(qsgw_ctx* ctx, int64_t nbf, int64_t nocc, const double* eps,
                      const double* diag, const float* mean, const float* scale, float* X);

/* y[b] = network(X[b]) for n states; X: [n][16], y: [n] FP32. */
int qsgw_mlp_forward(qsgw_ctx* ctx, const float* params, int64_t n, const float* X, float* y);

/*
 * BF16 inference of the same network (the learned warm start's inference
 * precision): X, W1, the first hidden activations, W2, the second hidden
 * activations and w3 are rounded to BF16 (nearest even) and multiplied on
 * the BF16 matrix cores with FP32 accumulation; biases and GELU stay FP32.
 * Same arguments and layout as qsgw_mlp_forward; FP32 master weights in.
 */
int qsgw_mlp_forward_bf16(qsgw_ctx* ctx, const float* params, int64_t n, const float* X, float* y);

/*
 * One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the
 * step count `step` >= 1, learning rate lr) on the mean squared error
 * L = (1/n) sum_b (network(X[b]) - target[b])^2 of a batch of n states.
 * params, adam_m, adam_v: [QSGW_MLP_NPARAMS] FP32, updated in place.
 * grad: NULL, or [QSGW_MLP_NPARAMS] FP32 out: dL/dparams before the update.
 * loss: NULL, or a device double out: L before the update.
 */
int qsgw_mlp_train_step(qsgw_ctx* ctx, float* params, float* adam_m, float* adam_v, int64_t step,
                        double lr, int64_t n, const float* X, const float* target, float* grad,
                        double* loss);

/*
 * Warm-start orbitals: eps = the values eps0[m] + delta[m] sorted ascending
 * (stable), C = C0 with its columns permuted the same way.  eps0, eps: [nbf]
 * FP64; delta: [nbf] FP32; C0, C: [nbf][nbf] FP64 (must not alias).
 */
int qsgw_warm_start(qsgw_ctx* ctx, int64_t nbf, const double* eps0, const double* C0,
                    const float* delta, double* eps, double* C);

#ifdef __cplusplus
}
#endif

#endif /* QSGW_H */
