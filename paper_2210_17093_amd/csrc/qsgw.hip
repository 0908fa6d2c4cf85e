// C-ABI of libqsgw: stage drivers and the single-problem qsGW iteration.
// Every numerical step runs in the kernels of this library (FP64/FP32
// matrix-core GEMMs of gemm_f64.hpp and the plain kernels of kernels.hip); the
// dense symmetric eigensolves go to rocSOLVER and are timed apart.
#include "internal.hpp"

namespace {


// Near-pole columns of the reduced-precision qsGW product for one excitation
// block: for each 64-row tile t of m, the (k, s) with Omega_s inside the
// window where some m of the tile may be within thr of a pole (k_near_ranges),
// compacted into ktab / stab at base_h[t] (tot_h[t] columns).
struct NearLists {
  int64_t *lo = nullptr, *cnt = nullptr;  // device [ntiles][nbf]: the s range of (t, k)
  const int32_t *ktab = nullptr, *stab = nullptr;
  std::vector<int64_t> tot_h, base_h;
  int64_t lmax = 0, ltot = 0, nt = 0;
};

int near_lists(qsgw_ctx* c, int64_t nbf, int64_t nocc, int64_t ns, const double* eps,
               const double* Omega, double thr, NearLists* nl) {
  const int64_t nt = (nbf + 63) / 64;
  int64_t* nearws = nullptr;
  CHECK(ws_get(c, W_NEAR, (size_t)(3 * nt * nbf + 2 * nt), &nearws));
  int64_t *lo = nearws, *cnt = lo + nt * nbf, *off = cnt + nt * nbf, *tot = off + nt * nbf,
          *base = tot + nt;
  hipLaunchKernelGGL(k_near_ranges, dim3(blocks_for(nt * nbf)), dim3(256), 0, c->stream, eps, Omega,
                     nbf, nocc, ns, thr, nt, lo, cnt);
  hipLaunchKernelGGL(k_near_offsets, dim3((unsigned)nt), dim3(256), 0, c->stream, cnt, nbf, nt, off,
                     tot, base);
  hipLaunchKernelGGL(k_near_bases, dim3(1), dim3(64), 0, c->stream, tot, nt, base);
  CHECK(launch_check(c, "near-pole ranges"));
  nl->tot_h.assign(nt, 0);
  nl->base_h.assign(nt, 0);
  HIP_TRY(c, hipMemcpyAsync(nl->tot_h.data(), tot, nt * sizeof(int64_t), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(nl->base_h.data(), base, nt * sizeof(int64_t), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  nl->lmax = nl->ltot = 0;
  for (int64_t t = 0; t < nt; ++t) {
    nl->lmax = nl->tot_h[t] > nl->lmax ? nl->tot_h[t] : nl->lmax;
    nl->ltot += nl->tot_h[t];
  }
  int32_t* tab = nullptr;
  CHECK(ws_get(c, W_NEARTAB, (size_t)(2 * nl->ltot + 2), &tab));
  if (nl->ltot > 0) {
    hipLaunchKernelGGL(k_near_fill, dim3((unsigned)(nt * nbf)), dim3(256), 0, c->stream, lo, cnt,
                       off, base, nbf, nt, tab, tab + nl->ltot + 1);
    CHECK(launch_check(c, "k_near_fill"));
  }
  nl->lo = lo;
  nl->cnt = cnt;
  nl->ktab = tab;
  nl->stab = tab + nl->ltot + 1;
  nl->nt = nt;
  return QSGW_OK;
}

// Split-BF16 operands of the qsGW product for one excitation block, written by
// the residue epilogue (EpiPairResidueX3): w and its pole-weighted copy in the
// Split8 layout, rows m < nbf of cs, k index j = k * nsp + s, K padded with
// zero chunks to kfar (a multiple of 32).
struct X3Out {
  uint16_t* ws;
  uint16_t* whs;
  int64_t cs, nsp, kfar;
  int64_t plane() const { return kfar * cs; }
  // exact near-pole terms (near_x3): compacted (k, s) columns and, per (m, k),
  // the near-pole excitations slo .. slo + len - 1 at columns c0 ..
  const int32_t* colidx;  // [nbf][nsp], -1 where not near any m
  const int32_t *c0, *slo, *len;  // [nbf][nbf]
  float* wN;  // [ncols][nbf] FP32 residues of the columns
  int64_t ncols;
};

// The exact near-pole terms of one excitation block (|x_mks| < thr), listed
// before the residue product so that its epilogue can keep the FP32 residues
// of those (k, s) columns, compacted.
int near_x3(qsgw_ctx* c, int64_t nbf, int64_t nocc, int64_t ns, const double* eps,
            const double* Omega, double thr, X3Out* x) {
  const int64_t nsp = x->nsp, nn = nbf * nbf;
  int64_t* iw = nullptr;
  CHECK(ws_get(c, W_NEAR, (size_t)(2 * nbf * nsp + 2 * nbf), &iw));
  int64_t *flag = iw, *off = flag + nbf * nsp, *total = off + nbf * nsp, *base = total + nbf;
  int32_t* tw = nullptr;
  CHECK(ws_get(c, W_NEARTAB, (size_t)(nbf * nsp + 3 * nn), &tw));
  int32_t *colidx = tw, *c0 = tw + nbf * nsp, *slo = c0 + nn, *len = slo + nn;
  hipLaunchKernelGGL(k_near_colflags, dim3(blocks_for(nbf * nsp)), dim3(256), 0, c->stream, eps,
                     Omega, nbf, nocc, ns, nsp, thr, flag);
  hipLaunchKernelGGL(k_near_offsets, dim3((unsigned)nbf), dim3(256), 0, c->stream, flag, nsp, nbf,
                     off, total, base);
  hipLaunchKernelGGL(k_near_bases, dim3(1), dim3(64), 0, c->stream, total, nbf, base);
  CHECK(launch_check(c, "near-pole columns"));
  int64_t tail[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(&tail[0], base + nbf - 1, sizeof(int64_t), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(&tail[1], total + nbf - 1, sizeof(int64_t), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  x->ncols = tail[0] + tail[1];
  if (x->ncols >= ((int64_t)1 << 31)) return fail(c, QSGW_ERR_UNSUPPORTED, "too many near-pole columns");
  hipLaunchKernelGGL(k_near_colidx, dim3(blocks_for(nbf * nsp)), dim3(256), 0, c->stream, flag, off,
                     base, nbf, nsp, colidx);
  hipLaunchKernelGGL(k_near_mk, dim3(blocks_for(nn)), dim3(256), 0, c->stream, eps, Omega, nbf, nocc,
                     ns, nsp, thr, colidx, c0, slo, len);
  CHECK(launch_check(c, "near-pole terms"));
  CHECK(ws_get(c, W_NEARW, (size_t)(x->ncols * nbf), &x->wN));
  x->colidx = colidx;
  x->c0 = c0;
  x->slo = slo;
  x->len = len;
  return QSGW_OK;
}

// ------------------------------------------------------------- stages ----

// Eq. (16): T = B_ao C (one GEMM over all P), B_mo[P] = C^T T[P] (batched
// over P, upper tiles only, mirrored).  CT is the matrix-core type.
template <class CT>
int stage_mo_transform_t(qsgw_ctx* c, int64_t nbf, int64_t naux, const double* B_ao,
                         const double* C, double* T, double* B_mo, Spans* sp,
                         float* B_mo32 = nullptr) {
  const int64_t nn = nbf * nbf;
  constexpr int BKm = std::is_same<CT, Bf16x3>::value ? 32 : 16;  // (k tile of the instruction)
  {
    Strided<true> A{B_ao, nbf, 1, 0, naux * nbf};
    Strided<false> B{C, 1, nbf, 0, nbf};
    EpiStore E{T, nbf, 0, 0, 1.0};
    E.nt = true;
    SPAN_OPEN(sp, kKMo1);
    CHECK((gemm_shape<CT, false, BKm>(c, c->tiles.shape[TU_MO1], "mo_transform/1", A, B, E, naux * nbf,
                                 nbf, nbf, 1)));
    SPAN_CLOSE(sp);
  }
  {
    Strided<false> A{C, 1, nbf, 0, nbf};
    Strided<false> B{T, 1, nbf, nn, nbf};
    EpiStore E{B_mo, nbf, nn, 0, 1.0};
    E.c32 = B_mo32;  // FP32 copy for the residue product of the FP32 variant
    SPAN_OPEN(sp, kKMo2);
    CHECK((gemm_shape<CT, true, BKm>(c, c->tiles.shape[TU_MO2], "mo_transform/2", A, B, E, nbf, nbf, nbf,
                                naux)));
    SPAN_CLOSE(sp);
  }
  return QSGW_OK;
}

int stage_mo_transform(qsgw_ctx* c, int64_t nbf, int64_t naux, const double* B_ao,
                       const double* C, double* T, double* B_mo, Spans* sp = nullptr,
                       int prec = QSGW_PREC_FP64, float* B_mo32 = nullptr) {
  // The split-BF16 variant transforms on the FP32 matrix cores: B_mo feeds
  // every later product and the Casida eigenvalues, and its split-BF16 error
  // grows with N_b (measured: 0.12 -> 0.52 meV of QP error at N_b = 600 for
  // 0.4 ms saved at N_b = 300).
  if (prec != QSGW_PREC_FP64)
    return stage_mo_transform_t<float>(c, nbf, naux, B_ao, C, T, B_mo, sp, B_mo32);
  return stage_mo_transform_t<double>(c, nbf, naux, B_ao, C, T, B_mo, sp);
}

// Eqs. (12)-(14): Delta, sqrt(Delta), Bt = B_ia sqrt(Delta), M = Delta^2 + 4 Bt^T Bt.
// Delta and sqrt(Delta) are always FP64; the product runs on the type of prec.
int stage_rpa_build(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                    const double* eps, double* M, double* sqrt_delta, double* delta, double* Bt,
                    int* flags, Spans* sp = nullptr, int prec = QSGW_PREC_FP64) {
  // The reduced-precision variants also keep Bt rounded to FP32 (W_BT32) for
  // their products.
  float* Bt32 = nullptr;
  if (prec == QSGW_PREC_FP32) {
    const int64_t n32 = naux * nocc * (nbf - nocc);
    CHECK(ws_get(c, W_BT32, (size_t)n32, &Bt32));
  }
  const int64_t nv = nbf - nocc, ntr = nocc * nv;
  SPAN_OPEN(sp, kKCasida);
  hipLaunchKernelGGL(k_transitions, dim3(blocks_for(ntr)), dim3(256), 0, c->stream, eps, nocc, nv,
                     delta, sqrt_delta, flags);
  CHECK(launch_check(c, "k_transitions"));
  hipLaunchKernelGGL(k_gather_bia, dim3(blocks_for(naux * ntr)), dim3(256), 0, c->stream, B_mo,
                     sqrt_delta, naux, nbf, nocc, Bt, Bt32);
  CHECK(launch_check(c, "k_gather_bia"));
  EpiCasida E{M, delta, ntr};
  if (prec == QSGW_PREC_FP32) {
    Strided<false, float> A{Bt32, 1, ntr, 0, ntr};
    CHECK((gemm_shape<float, true, 32>(c, c->tiles.shape[TU_CASIDA], "rpa_build", A, A, E, ntr,
                                       ntr, naux, 1)));
  } else if (prec == QSGW_PREC_SPLIT_BF16) {
    // Bt split once into BF16 halves in k-blocks of 8 (rows t, k = P)
    const int64_t kpad = (naux + 31) / 32 * 32, rp = (ntr + 127) / 128 * 128;
    uint16_t* bs = nullptr;
    CHECK(ws_get(c, W_SPLIT_CAS, (size_t)(2 * kpad * rp), &bs));
    hipLaunchKernelGGL(k_split_cols, dim3(blocks_for(rp * (kpad / 8))), dim3(256), 0, c->stream, Bt,
                       ntr, ntr, naux, rp, kpad, bs);
    CHECK(launch_check(c, "k_split_cols"));
    Split8 A{bs, rp, kpad * rp, 0};
    CHECK((gemm_shape<Bf16x3, true, 32>(c, c->tiles.shape[TU_CASIDA], "rpa_build", A, A, E, ntr,
                                        ntr, kpad, 1)));
  } else {
    Strided<false> A{Bt, 1, ntr, 0, ntr};
    CHECK((gemm_shape<double, true>(c, c->tiles.shape[TU_CASIDA], "rpa_build", A, A, E, ntr, ntr,
                                    naux, 1)));
  }
  SPAN_CLOSE(sp);
  return QSGW_OK;
}

int stage_rpa_solve(qsgw_ctx* c, int64_t ntr, double* M, double* Omega) {
  CHECK(eig_casida(c, ntr, M, Omega, "rpa_solve"));
  int* flags = nullptr;
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  HIP_TRY(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL(k_omega_from_eigs, dim3(blocks_for(ntr)), dim3(256), 0, c->stream, Omega, ntr,
                     Omega, flags);
  CHECK(launch_check(c, "k_omega_from_eigs"));
  int bad = 0;
  CHECK(read_flag(c, flags, &bad));
  if (bad) return fail(c, QSGW_ERR_SOLVER, "RPA instability: a Casida eigenvalue Omega^2 <= 0");
  return QSGW_OK;
}

// Casida eigensolve through the two-stage projection (Eq. (12)): Omega and
// rho'[P][s] = sqrt(2/Omega_s) sum_t Bt[P][t] Z[t][s] for every excitation
// (row-major [naux][ntr]), the rho' of Eq. (18), without forming Z.  M is
// destroyed; X is an [naux][ntr] work array.
int stage_rpa_solve_project(qsgw_ctx* c, int64_t ntr, int64_t naux, double* M, double* Omega,
                            const double* Bt, double* X, double* rho) {
  CHECK(eig_two_stage_project(c, ntr, M, Omega, naux, Bt, X, rho, "rpa_solve"));
  int* flags = nullptr;
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  HIP_TRY(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL(k_omega_from_eigs, dim3(blocks_for(ntr)), dim3(256), 0, c->stream, Omega, ntr,
                     Omega, flags);
  CHECK(launch_check(c, "k_omega_from_eigs"));
  int bad = 0;
  CHECK(read_flag(c, flags, &bad));
  if (bad) return fail(c, QSGW_ERR_SOLVER, "RPA instability: a Casida eigenvalue Omega^2 <= 0");
  hipLaunchKernelGGL(k_scale_rho, dim3(blocks_for(naux * ntr)), dim3(256), 0, c->stream, rho, naux,
                     ntr, Omega);
  return launch_check(c, "k_scale_rho");
}

// Eq. (18) for excitations [s0, s0 + ns): rho' = sqrt(2/Omega) Bt Z^T, w = B_mo^T rho'.
template <class CT>
int stage_residues_t(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t ntr, const double* B_mo,
                     const double* Bt, const double* Z, const double* Omega, int64_t s0, int64_t ns,
                     double* rho, double* w, Spans* sp, double* wh, const double* eps, int64_t nocc,
                     double eta, float* wh32 = nullptr, float* w32 = nullptr, double thr = 0.0,
                     const float* B_mo32 = nullptr, const float* Bt32_in = nullptr,
                     bool reuse_split = false, const X3Out* x3o = nullptr,
                     bool rho_ready = false, int64_t rho_ld = 0,
                     const float* rho32_in = nullptr) {
  // rho_ready: rho already holds rho' of this block (computed for another MO
  // tensor with the same Bt and Z, or by the eigensolver's projection), row P
  // at rho + P * rho_ld (rho_ld 0: ns), so only the w product runs; the FP32
  // variant then reads rho32_in (same layout) and the split-BF16 variant
  // splits rho.  Z is not read.
  // The FP32 variant reads FP32 copies of B_mo and rho' in the residue
  // product (half the operand bytes); rounding them is what its matrix cores
  // do anyway.  The split-BF16 variant reads them split into BF16 halves in
  // k-blocks of 8 (the same bytes), made once per B_mo (reuse_split: the
  // split of B_mo made for an earlier block of the same iteration is current).
  constexpr bool f32 = !std::is_same<CT, double>::value;
  constexpr bool x3 = std::is_same<CT, Bf16x3>::value;
  float* rho32 = nullptr;
  const float* Bt32 = Bt32_in;
  float* Z32 = nullptr;
  const int64_t kpad = ((naux + 31) / 32) * 32, ns_pad = ((ns + 127) / 128) * 128;
  const int32_t* blocks = nullptr;
  int64_t nblk = 0;
  CHECK(pair_blocks(c, nbf, &blocks, &nblk));
  uint16_t *splitA = nullptr, *splitB = nullptr;
  if (x3) {
    CHECK(ws_get(c, W_SPLIT_A, (size_t)(2 * kpad * nblk * 128), &splitA));
    CHECK(ws_get(c, W_SPLIT_B, (size_t)(2 * kpad * ns_pad), &splitB));
    if (!reuse_split) {  // (stage time; the kernel spans time the products alone)
      hipLaunchKernelGGL(k_split_pairs, dim3(blocks_for(nblk * 128 * (kpad / 8))), dim3(256), 0,
                         c->stream, B_mo, blocks, nblk, nbf, naux, kpad, splitA);
      CHECK(launch_check(c, "k_split_pairs"));
    }
  }
  uint16_t *splitRA = nullptr, *splitZ = nullptr;
  const int64_t kpt = ((ntr + 31) / 32) * 32, naux_pad = ((naux + 127) / 128) * 128;
  const int64_t ldr = rho_ld > 0 ? rho_ld : ns;
  if (x3 && !rho_ready) {
    // rho' = Bt Z^T from split copies: Bt with rows P (once per B_mo, as the
    // pair rows), the block's eigenvectors with rows s; k = t, padded to 32
    CHECK(ws_get(c, W_SPLIT_RA, (size_t)(2 * kpt * naux_pad), &splitRA));
    CHECK(ws_get(c, W_SPLIT_Z, (size_t)(2 * kpt * ns_pad), &splitZ));
    if (!reuse_split) {
      hipLaunchKernelGGL(k_split_rows, dim3((unsigned)(naux_pad / 32), (unsigned)((kpt + 255) / 256)),
                         dim3(256), 0, c->stream, Bt, ntr, naux, ntr, naux_pad, kpt, splitRA);
      CHECK(launch_check(c, "k_split_rows"));
    }
    hipLaunchKernelGGL(k_split_rows, dim3((unsigned)(ns_pad / 32), (unsigned)((kpt + 255) / 256)),
                       dim3(256), 0, c->stream, Z + s0 * ntr, ntr, ns, ntr, ns_pad, kpt, splitZ);
    CHECK(launch_check(c, "k_split_rows"));
  } else if (f32 && !x3) {
    if (!rho_ready) {
      if (!Bt32) {
        float* b = nullptr;
        CHECK(ws_get(c, W_BT32, (size_t)(naux * ntr), &b));
        hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(naux * ntr)), dim3(256), 0, c->stream, Bt,
                           naux * ntr, b);
        CHECK(launch_check(c, "k_to_f32"));
        Bt32 = b;
      }
      CHECK(ws_get(c, W_Z32, (size_t)(ns * ntr), &Z32));
      hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(ns * ntr)), dim3(256), 0, c->stream,
                         Z + s0 * ntr, ns * ntr, Z32);
      CHECK(launch_check(c, "k_to_f32"));
      CHECK(ws_get(c, W_RHO32, (size_t)(naux * ns), &rho32));
    } else {
      if (!rho32_in) return fail(c, QSGW_ERR_INVALID_ARG, "residues: no FP32 copy of rho'");
      rho32 = const_cast<float*>(rho32_in);
    }
    if (!B_mo32) {
      float* b32 = nullptr;
      CHECK(ws_get(c, W_BMO32, (size_t)(naux * nbf * nbf), &b32));
      hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(naux * nbf * nbf)), dim3(256), 0, c->stream, B_mo,
                         naux * nbf * nbf, b32);
      CHECK(launch_check(c, "k_to_f32"));
      B_mo32 = b32;
    }
  }
  if (!rho_ready) {
    const int64_t maxk = f32 ? kFp32MaxK : ntr;
    const int64_t kr = x3 ? kpt : ntr;  // (k length of the product)
    SplitPlan spl = rho_split(c->tiles, naux, ns, kr, maxk);
    if (f32) spl = round_chunks(spl, kr, 32);
    auto rho_gemm = [&](auto E, SplitPlan p) -> int {
      if constexpr (x3) {
        Split8 A{splitRA, naux_pad, kpt * naux_pad, 0};
        Split8 B{splitZ, ns_pad, kpt * ns_pad, 0};
        return gemm_shape<CT, false, 32>(c, c->tiles.shape[TU_RHO], "residues/rho", A, B, E, naux,
                                         ns, kpt, 1, p);
      } else if constexpr (f32) {
        Strided<true, float> A{Bt32, ntr, 1, 0, naux};
        Strided<true, float> B{Z32, ntr, 1, 0, ns};
        return gemm_shape<CT, false, 32>(c, c->tiles.shape[TU_RHO], "residues/rho", A, B, E, naux,
                                         ns, ntr, 1, p);
      } else {
        Strided<true> A{Bt, ntr, 1, 0, naux};
        Strided<true> B{Z + s0 * ntr, ntr, 1, 0, ns};
        return gemm_shape<CT, false>(c, c->tiles.shape[TU_RHO], "residues/rho", A, B, E, naux, ns,
                                     ntr, 1, p);
      }
    };
    SPAN_OPEN(sp, kKRho);
    if (spl.nz > 1) {
      double* part = nullptr;
      CHECK(ws_get(c, W_RHOPART, (size_t)(spl.nz * naux * ns), &part));
      EpiStore E{part, ns, 0, naux * ns, 1.0};
      CHECK(rho_gemm(E, spl));
      hipLaunchKernelGGL(k_rho_reduce, dim3(blocks_for(naux * ns)), dim3(256), 0, c->stream, part,
                         spl.nz, naux, ns, Omega + s0, rho, rho32);
      CHECK(launch_check(c, "k_rho_reduce"));
    } else {
      EpiRho E{rho, Omega + s0, ns};
      E.rho32 = rho32;
      CHECK(rho_gemm(E, SplitPlan{0, 1}));
    }
    SPAN_CLOSE(sp);
  }
  if (x3) {
    hipLaunchKernelGGL(k_split_cols, dim3(blocks_for(ns_pad * (kpad / 8))), dim3(256), 0, c->stream,
                       rho, ldr, ns, naux, ns_pad, kpad, splitB);
    CHECK(launch_check(c, "k_split_cols"));
  }
  {
    const int64_t nn = nbf * nbf;
    EpiPairResidue E{w, wh, blocks, eps, Omega + s0, nbf, nocc, ns, eta};
    E.wh32 = wh32;
    E.w32 = w32;
    E.thr = thr;
    SPAN_OPEN(sp, kKW);
    if constexpr (x3) {
      const int64_t rows = nblk * 128;
      Split8 A{splitA, rows, kpad * rows, 0};
      Split8 B{splitB, ns_pad, kpad * ns_pad, 0};
      if (x3o) {
        EpiPairResidueX3 E3{w,      x3o->wN,      x3o->colidx, x3o->ws, x3o->whs,
                            x3o->cs, x3o->plane(), x3o->nsp,   blocks,  eps,
                            Omega + s0, nbf,       nocc,        ns,      eta,
                            thr};
        CHECK((gemm_t<CT, 128, 128, false, 32>(c, "residues/w", A, B, E3, rows, ns, kpad, 1)));
      } else {
        CHECK((gemm_t<CT, 128, 128, false, 32>(c, "residues/w", A, B, E, rows, ns, kpad, 1)));
      }
    } else if constexpr (f32) {
      // k tiles of 32: twice the matrix-core work per barrier and per prefetch
      PairRows<8, 16, float> A{B_mo32, nn, 0, nbf, blocks};
      Strided<false, float> B{rho32, 1, ldr, 0, ns};
      CHECK((gemm_t<CT, 128, 128, false, 32>(c, "residues/w", A, B, E, nblk * 128, ns, naux, 1)));
    } else {
      PairRows<8, 16> A{B_mo, nn, 0, nbf, blocks};
      Strided<false> B{rho, 1, ldr, 0, ns};
      CHECK((gemm_t<CT, 128, 128, false>(c, "residues/w", A, B, E, nblk * 128, ns, naux, 1)));
    }
    SPAN_CLOSE(sp);
  }
  return QSGW_OK;
}

int stage_residues(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t ntr, const double* B_mo,
                   const double* Bt, const double* Z, const double* Omega, int64_t s0, int64_t ns,
                   double* rho, double* w, Spans* sp = nullptr, double* wh = nullptr,
                   const double* eps = nullptr, int64_t nocc = 0, double eta = 0.0,
                   int prec = QSGW_PREC_FP64, float* wh32 = nullptr, float* w32 = nullptr,
                   double thr = 0.0, const float* B_mo32 = nullptr, const float* Bt32 = nullptr,
                   bool reuse_split = false, const X3Out* x3o = nullptr,
                   bool rho_ready = false, int64_t rho_ld = 0, const float* rho32 = nullptr) {
  if (prec == QSGW_PREC_FP32)
    return stage_residues_t<float>(c, nbf, naux, ntr, B_mo, Bt, Z, Omega, s0, ns, rho, w, sp, wh,
                                   eps, nocc, eta, wh32, w32, thr, B_mo32, Bt32, false, nullptr,
                                   rho_ready, rho_ld, rho32);
  if (prec == QSGW_PREC_SPLIT_BF16)
    return stage_residues_t<Bf16x3>(c, nbf, naux, ntr, B_mo, Bt, Z, Omega, s0, ns, rho, w, sp, wh,
                                    eps, nocc, eta, wh32, w32, thr, B_mo32, Bt32, reuse_split, x3o,
                                    rho_ready, rho_ld);
  return stage_residues_t<double>(c, nbf, naux, ntr, B_mo, Bt, Z, Omega, s0, ns, rho, w, sp, wh,
                                  eps, nocc, eta, nullptr, nullptr, 0.0, nullptr, nullptr, false,
                                  nullptr, rho_ready, rho_ld);
}

// Reduced-precision variant of Eq. (19) for one excitation block (PT: float
// for FP32 matrix-core products, Bf16x3 for split-BF16).  G = G_far + G_near:
// G_far = Wh32 W32^T over every term with |x| >= thr (FP32 matrix cores,
// FP64 split-K reduction); G_near over the near-pole terms (|x| < thr) in
// FP64, for each 64-row tile of m over the compacted (k, s) columns in
// which some m of the tile is near a pole.  V (+)= 1/2 (G + G^T).
template <class PT>
int stage_sigma_qs32_t(qsgw_ctx* c, int64_t nbf, int64_t nocc, int64_t ns, const float* wh32,
                       const float* w32, const double* eps, const double* Omega, double eta,
                       double thr, double* V, int accumulate, Spans* spn,
                       const X3Out* x3o = nullptr) {
  // (split-BF16 with split operands: the far product runs over the padded k
  // index of the Split8 layout, kfar >= nbf * ns)
  const int64_t nn = nbf * nbf, K = x3o ? x3o->kfar : nbf * ns, nt = (nbf + 63) / 64;
  if (K >= (int64_t)1 << 31) return fail(c, QSGW_ERR_INVALID_ARG, "sigma: nbf * ns must stay below 2^31");
  SplitPlan spf = sigma_split32(c->tiles, nbf, K);
  if (spf.nz > 1) {  // the far product runs k tiles of 32: chunks are multiples of 32
    spf.kchunk = ((spf.kchunk + 31) / 32) * 32;
    spf.nz = (K + spf.kchunk - 1) / spf.kchunk;
  }
  NearLists nl;
  SPAN_OPEN(spn, kKSigma);
  int64_t zn = near_slices_max(nbf);
  double* part = nullptr;
  double* npart = nullptr;
  if (x3o) {
    // exact near-pole terms from the compacted FP32 columns, k in slices of kc
    const int64_t kc = kX3NearK;
    zn = x3_near_slices(nbf);
    if (nbf > 2048) return fail(c, QSGW_ERR_UNSUPPORTED, "split-BF16 near-pole part: nbf > 2048");
    CHECK(ws_get(c, W_PART, (size_t)((spf.nz + zn) * nn), &part));
    npart = part + spf.nz * nn;
    hipLaunchKernelGGL(k_near_product, dim3((unsigned)nbf, (unsigned)zn), dim3(256), 0, c->stream,
                       eps, Omega, nbf, nocc, eta, x3o->c0, x3o->slo, x3o->len, x3o->wN, kc,
                       npart);
    CHECK(launch_check(c, "k_near_product"));
  } else {
    CHECK(near_lists(c, nbf, nocc, ns, eps, Omega, thr, &nl));
    const int64_t zcap = (nl.lmax + 255) / 256;
    if (zn > zcap) zn = zcap < 1 ? 1 : zcap;
    CHECK(ws_get(c, W_PART, (size_t)((spf.nz + zn) * nn), &part));
    npart = part + spf.nz * nn;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(zn * nn)), dim3(256), 0, c->stream, npart, zn * nn,
                       0.0);
    CHECK(launch_check(c, "k_fill"));
  }
  const std::vector<int64_t>& tot_h = nl.tot_h;
  const std::vector<int64_t>& base_h = nl.base_h;
  const int32_t *ktab = nl.ktab, *stab = nl.stab;
  if constexpr (std::is_same<PT, Bf16x3>::value) {
    if (x3o) {
      // zero k chunks beyond nbf * nsp (the residue epilogue writes the rest)
      const int64_t kb0 = nbf * x3o->nsp / 8, tail = (x3o->kfar / 8 - kb0) * x3o->cs * 8;
      if (tail > 0) {
        uint16_t* t[4] = {x3o->ws, x3o->ws + x3o->plane(), x3o->whs, x3o->whs + x3o->plane()};
        for (uint16_t* q : t) {
          hipLaunchKernelGGL(k_zero_u16, dim3(blocks_for(tail)), dim3(256), 0, c->stream,
                             q + kb0 * x3o->cs * 8, tail);
        }
        CHECK(launch_check(c, "k_zero_u16"));
      }
      Split8 A{x3o->whs, x3o->cs, x3o->plane(), 0};
      Split8 B{x3o->ws, x3o->cs, x3o->plane(), 0};
      EpiStore E{part, nbf, 0, nn, 1.0};
      switch (c->tiles.shape[TU_SIGMA]) {
        case SH_64x64:
          CHECK((gemm_t<PT, 64, 64, false, 32>(c, "sigma_qs/far", A, B, E, nbf, nbf, K, 1, spf)));
          break;
        case SH_128x128:
          CHECK((gemm_t<PT, 128, 128, false, 32>(c, "sigma_qs/far", A, B, E, nbf, nbf, K, 1, spf)));
          break;
        default:
          CHECK((gemm_t<PT, 128, 64, false, 32>(c, "sigma_qs/far", A, B, E, nbf, nbf, K, 1, spf)));
      }
    }
  }
  if (!x3o) {
    Strided<true, float> A{wh32, K, 1, 0, nbf};
    Strided<true, float> B{w32, K, 1, 0, nbf};
    EpiStore E{part, nbf, 0, nn, 1.0};
    const SplitPlan sp32 = spf;  // chunks are multiples of 32 (see above)
    switch (c->tiles.shape[TU_SIGMA]) {
      case SH_64x64:
        CHECK((gemm_t<PT, 64, 64, false, 32>(c, "sigma_qs/far", A, B, E, nbf, nbf, K, 1, sp32)));
        break;
      case SH_128x128:
        CHECK((gemm_t<PT, 128, 128, false, 32>(c, "sigma_qs/far", A, B, E, nbf, nbf, K, 1, sp32)));
        break;
      default:
        CHECK((gemm_t<PT, 128, 64, false, 32>(c, "sigma_qs/far", A, B, E, nbf, nbf, K, 1, sp32)));
    }
  }
  for (int64_t t = 0; t < (x3o ? 0 : nt); ++t) {
    const int64_t L = tot_h[t];
    if (L == 0) continue;
    const int64_t m0 = t * 64, rows = (m0 + 64 < nbf ? 64 : nbf - m0);
    int64_t kchunk = (L + zn - 1) / zn;
    kchunk = ((kchunk + 15) / 16) * 16;
    NearRowsOp A{w32, eps, Omega, ktab + base_h[t], stab + base_h[t], m0, rows, nbf, nocc, ns, eta,
                 thr};
    NearColsOp B{w32, ktab + base_h[t], stab + base_h[t], nbf, ns};
    EpiStore E{npart + m0 * nbf, nbf, 0, nn, 1.0};
    CHECK((gemm_t<double, 64, 64, false>(c, "sigma_qs/near", A, B, E, rows, nbf, L, 1,
                                         SplitPlan{kchunk, zn})));
  }
  SPAN_CLOSE(spn);
  SPAN_OPEN(spn, kKSigmaRed);
  CHECK(reduce_sym(c, part, spf.nz + zn, nbf, V, accumulate));
  SPAN_CLOSE(spn);
  return QSGW_OK;
}

// Eq. (19) contribution of one excitation block: V (+)= 1/2 (G + G^T).
int stage_sigma_qs(qsgw_ctx* c, int64_t nbf, int64_t nocc, int64_t ns, const double* w,
                   const double* eps, const double* Omega, double eta, double* V, int accumulate,
                   Spans* spn = nullptr, const double* wh = nullptr) {
  const SplitPlan sp = sigma_split(c->tiles, nbf, ns);
  if (nbf * ns >= (int64_t)1 << 32)
    return fail(c, QSGW_ERR_INVALID_ARG, "sigma: nbf * ns must stay below 2^32");
  double* part = nullptr;
  CHECK(ws_get(c, W_PART, (size_t)(sp.nz * nbf * nbf), &part));
  Strided<true> B{w, nbf * ns, 1, 0, nbf};
  EpiStore E{part, nbf, 0, nbf * nbf, 1.0};
  SPAN_OPEN(spn, kKSigma);
  if (wh) {
    // pole weights already applied by the residue epilogue
    Strided<true> A{wh, nbf * ns, 1, 0, nbf};
    CHECK((gemm_shape<double, false>(c, c->tiles.shape[TU_SIGMA], "sigma_qs", A, B, E, nbf, nbf,
                                     nbf * ns, 1, sp)));
  } else {
    PoleScaledResidueOp A{w, eps, Omega, nbf, nocc, ns, eta};
    CHECK((gemm_shape<double, false>(c, c->tiles.shape[TU_SIGMA], "sigma_qs", A, B, E, nbf, nbf,
                                     nbf * ns, 1, sp)));
  }
  SPAN_CLOSE(spn);
  SPAN_OPEN(spn, kKSigmaRed);
  CHECK(reduce_sym(c, part, sp.nz, nbf, V, accumulate));
  SPAN_CLOSE(spn);
  return QSGW_OK;
}

// Hartree and exchange in the MO basis of the orbitals that produced B_mo:
// J = 2 sum_P c_P B^P, c_P = sum_i B^P_ii;  K = sum_P B^P_{:,occ} (B^P_{:,occ})^T.
// Leaves J in W_J and the K partial sums in W_PART; returns their count.
int stage_jk_mo(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                double** J, double** Kpart, int64_t* nz) {
  const int64_t nn = nbf * nbf;
  double* cp = nullptr;
  CHECK(ws_get(c, W_CP, (size_t)naux, &cp));
  CHECK(ws_get(c, W_J, (size_t)nn, J));
  hipLaunchKernelGGL(k_occ_trace, dim3(blocks_for(naux)), dim3(256), 0, c->stream, B_mo, naux, nbf,
                     nocc, cp);
  CHECK(launch_check(c, "k_occ_trace"));
  {
    // J over groups of 32 auxiliary functions (many threads, coalesced), then
    // the sum of the groups
    constexpr int64_t pg = 32;
    const int64_t ng = (naux + pg - 1) / pg;
    double* jp = nullptr;
    CHECK(ws_get(c, W_REDPART, (size_t)(ng * nn), &jp));
    hipLaunchKernelGGL(k_hartree_part, dim3(blocks_for(ng * nn)), dim3(256), 0, c->stream, B_mo,
                       cp, naux, nn, pg, jp);
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks_for(nn)), dim3(256), 0, c->stream, jp, ng, nn, ng,
                       *J);
    CHECK(launch_check(c, "k_hartree_part"));
  }
  const SplitPlan sp = exchange_split(c->tiles, nbf, naux, nocc);
  CHECK(ws_get(c, W_PART, (size_t)(sp.nz * nn), Kpart));
  OccRowsOp A{B_mo, nbf, nocc};
  EpiStore E{*Kpart, nbf, 0, nn, 1.0};
  CHECK((gemm_shape<double, true>(c, c->tiles.shape[TU_EXCHANGE], "exchange_mo", A, A, E, nbf, nbf,
                                  naux * nocc, 1, sp)));
  *nz = sp.nz;
  return QSGW_OK;
}

// out = X^T Y X for square n x n matrices (row-major):  tmp = Y X, out = X^T tmp.
int congruence_t(qsgw_ctx* c, int64_t n, const double* X, const double* Y, double* tmp,
                 double* out) {
  {
    Strided<true> A{Y, n, 1, 0, n};
    Strided<false> B{X, 1, n, 0, n};
    EpiStore E{tmp, n, 0, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "congruence/1", A, B, E, n, n, n, 1)));
  }
  {
    Strided<false> A{X, 1, n, 0, n};
    Strided<false> B{tmp, 1, n, 0, n};
    EpiStore E{out, n, 0, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "congruence/2", A, B, E, n, n, n, 1)));
  }
  return QSGW_OK;
}

// out = X Y X^T:  tmp = X Y, out = tmp X^T.
int congruence(qsgw_ctx* c, int64_t n, const double* X, const double* Y, double* tmp,
               double* out) {
  {
    Strided<true> A{X, n, 1, 0, n};
    Strided<false> B{Y, 1, n, 0, n};
    EpiStore E{tmp, n, 0, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "congruence/3", A, B, E, n, n, n, 1)));
  }
  {
    Strided<true> A{tmp, n, 1, 0, n};
    Strided<true> B{X, n, 1, 0, n};
    EpiStore E{out, n, 0, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "congruence/4", A, B, E, n, n, n, 1)));
  }
  return QSGW_OK;
}

int check_prec(qsgw_ctx* c, int precision) {
  if (precision == QSGW_PREC_FP64 || precision == QSGW_PREC_FP32 ||
      precision == QSGW_PREC_SPLIT_BF16)
    return QSGW_OK;
  return fail(c, QSGW_ERR_INVALID_ARG, "unknown precision %d", precision);
}


}  // namespace

// ================================================================ C-ABI ====
extern "C" {

int qsgw_version(void) { return QSGW_VERSION; }

int qsgw_ctx_create(qsgw_ctx** out, void* hip_stream) {
  if (!out) return QSGW_ERR_INVALID_ARG;
  *out = nullptr;
  qsgw_ctx* c = new (std::nothrow) qsgw_ctx();
  if (!c) return QSGW_ERR_ALLOC;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return QSGW_ERR_HIP;
  }
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
    delete c;
    return QSGW_ERR_SOLVER;
  }
  if (rocblas_set_stream(c->blas, c->stream) != rocblas_status_success) {
    rocblas_destroy_handle(c->blas);
    delete c;
    return QSGW_ERR_SOLVER;
  }
  // the allocation-free entry point reports a failed lookup itself
  if (noalloc_setup(c) != QSGW_OK) c->scratch = nullptr;
  c->err.clear();
  *out = c;
  return QSGW_OK;
}

int qsgw_ctx_destroy(qsgw_ctx* c) {
  if (!c) return QSGW_OK;
  (void)hipStreamSynchronize(c->stream);
  for (int i = 0; i < qsgw_ctx::kAux; ++i) {
    if (c->aux[i]) (void)hipStreamSynchronize(c->aux[i]);
    if (c->aux_blas[i]) rocblas_destroy_handle(c->aux_blas[i]);
    if (c->aux[i]) (void)hipStreamDestroy(c->aux[i]);
    if (c->join[i]) (void)hipEventDestroy(c->join[i]);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  for (auto& b : c->ws)
    if (b.p) (void)hipFree(b.p);
  for (auto e : c->events) (void)hipEventDestroy(e);
  if (c->blas) rocblas_destroy_handle(c->blas);
  delete c;
  return QSGW_OK;
}

const char* qsgw_last_error(const qsgw_ctx* c) { return c ? c->err.c_str() : "null context"; }

int qsgw_last_stage_ms(const qsgw_ctx* c0, double* ms, int n) {
  qsgw_ctx* c = const_cast<qsgw_ctx*>(c0);
  if (!c || !ms || n < 0) return QSGW_ERR_INVALID_ARG;
  if (c->last_stage >= 0 && c->events.size() >= 2) {
    HIP_TRY(c, hipEventSynchronize(c->events[1]));
    for (int i = 0; i < 7; ++i) c->stage_ms[i] = 0.0;
    c->stage_ms[c->last_stage] = elapsed(c, 0, 1);
  }
  for (int i = 0; i < n && i < 7; ++i) ms[i] = c->stage_ms[i];
  return QSGW_OK;
}

int qsgw_mo_transform(qsgw_ctx* c, int64_t nbf, int64_t naux, const double* B_ao, const double* C,
                      double* B_mo, int precision) {
  CHECK(check_common(c, nbf, naux));
  CHECK(check_prec(c, precision));
  if (!B_ao || !C || !B_mo) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  CHECK(check_finite(c, "qsgw_mo_transform", {fin(B_ao, naux * nbf * nbf, "B_ao"), fin(C, nbf * nbf, "C")}));
  double* T = nullptr;
  CHECK(ws_get(c, W_T, (size_t)(naux * nbf * nbf), &T));
  CHECK(single_begin(c, kStageMo));
  CHECK(stage_mo_transform(c, nbf, naux, B_ao, C, T, B_mo, nullptr, precision));
  return single_end(c);
}

int qsgw_rpa_build(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                   const double* eps, double* M, double* sqrt_delta, int precision) {
  CHECK(check_common(c, nbf, naux));
  CHECK(check_prec(c, precision));
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  if (!B_mo || !eps || !M || !sqrt_delta) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  CHECK(check_finite(c, "qsgw_rpa_build", {fin(B_mo, naux * nbf * nbf, "B_mo"), fin(eps, nbf, "eps")}));
  const int64_t ntr = nocc * (nbf - nocc);
  double *delta = nullptr, *Bt = nullptr;
  int* flags = nullptr;
  CHECK(ws_get(c, W_DELTA, (size_t)ntr, &delta));
  CHECK(ws_get(c, W_BT, (size_t)(naux * ntr), &Bt));
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  HIP_TRY(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
  CHECK(single_begin(c, kStageRpa));
  CHECK(stage_rpa_build(c, nbf, naux, nocc, B_mo, eps, M, sqrt_delta, delta, Bt, flags, nullptr,
                        precision));
  CHECK(single_end(c));
  int bad = 0;
  CHECK(read_flag(c, flags, &bad));
  if (bad) return fail(c, QSGW_ERR_INVALID_ARG, "eps[a] - eps[i] must be > 0 for every transition");
  return QSGW_OK;
}

int qsgw_rpa_solve(qsgw_ctx* c, int64_t ntr, double* M_to_Z, double* Omega) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (ntr < 1 || !M_to_Z || !Omega) return fail(c, QSGW_ERR_INVALID_ARG, "bad arguments");
  CHECK(check_finite(c, "qsgw_rpa_solve", {fin(M_to_Z, ntr * ntr, "M")}));
  CHECK(single_begin(c, kStageEigRpa));
  CHECK(stage_rpa_solve(c, ntr, M_to_Z, Omega));
  return single_end(c);
}

int qsgw_residues(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                  const double* sqrt_delta, const double* Z, const double* Omega, int64_t s_begin,
                  int64_t s_count, double* w, double* wh, const double* eps, double eta,
                  int precision) {
  CHECK(check_common(c, nbf, naux));
  CHECK(check_prec(c, precision));
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  const int64_t ntr = nocc * (nbf - nocc);
  if (s_begin < 0 || s_count < 1 || s_begin + s_count > ntr)
    return fail(c, QSGW_ERR_INVALID_ARG, "excitation range [%lld, %lld) outside [0, %lld)",
                (long long)s_begin, (long long)(s_begin + s_count), (long long)ntr);
  if (!B_mo || !sqrt_delta || !Z || !Omega || !w)
    return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  if (wh && (!eps || !(eta > 0.0) || !isfinite(eta)))
    return fail(c, QSGW_ERR_INVALID_ARG, "the pole-weighted copy needs eps and a finite eta > 0");
  CHECK(check_finite(c, "qsgw_residues",
                     {fin(B_mo, naux * nbf * nbf, "B_mo"), fin(sqrt_delta, ntr, "sqrt_delta"),
                      fin(Z, ntr * ntr, "Z"), fin(Omega, ntr, "Omega"),
                      fin(wh ? eps : nullptr, nbf, "eps")}));
  double *Bt = nullptr, *rho = nullptr;
  float* Bt32 = nullptr;
  CHECK(ws_get(c, W_BT, (size_t)(naux * ntr), &Bt));
  CHECK(ws_get(c, W_RHO, (size_t)(naux * s_count), &rho));
  if (precision != QSGW_PREC_FP64) CHECK(ws_get(c, W_BT32, (size_t)(naux * ntr), &Bt32));
  CHECK(single_begin(c, kStageRes));
  hipLaunchKernelGGL(k_gather_bia, dim3(blocks_for(naux * ntr)), dim3(256), 0, c->stream, B_mo,
                     sqrt_delta, naux, nbf, nocc, Bt, Bt32);
  CHECK(launch_check(c, "k_gather_bia"));
  CHECK(stage_residues(c, nbf, naux, ntr, B_mo, Bt, Z, Omega, s_begin, s_count, rho, w, nullptr,
                       wh, eps, nocc, eta, precision, nullptr, nullptr, 0.0, nullptr, Bt32));
  return single_end(c);
}

int qsgw_sigma(qsgw_ctx* c, int mode, int64_t nbf, int64_t nocc, int64_t ns, const double* w,
               const double* wh, const double* eps, const double* Omega, double eta,
               const double* omega, int64_t nomega, const int64_t* states, int64_t nstates,
               double* out, int accumulate) {
  CHECK(check_common(c, nbf, 1));
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  if (ns < 1) return fail(c, QSGW_ERR_INVALID_ARG, "need ns >= 1");
  if (!(eta > 0.0) || !isfinite(eta)) return fail(c, QSGW_ERR_INVALID_ARG, "need finite eta > 0");
  if (!w || !eps || !Omega || !out) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  CHECK(check_finite(c, "qsgw_sigma",
                     {fin(w, nbf * nbf * ns, "w"),
                      fin(mode == QSGW_SIGMA_QS_MATRIX ? wh : nullptr, nbf * nbf * ns, "wh"),
                      fin(eps, nbf, "eps"), fin(Omega, ns, "Omega"),
                      fin(mode == QSGW_SIGMA_DIAG_GRID ? omega : nullptr, nomega, "omega")}));
  if (mode == QSGW_SIGMA_QS_MATRIX) {
    CHECK(single_begin(c, kStageSigma));
    CHECK(stage_sigma_qs(c, nbf, nocc, ns, w, eps, Omega, eta, out, accumulate ? 1 : 0, nullptr,
                         wh));
    return single_end(c);
  }
  if (mode == QSGW_SIGMA_DIAG_SELF) {
    if (nstates < 1 || !states) return fail(c, QSGW_ERR_INVALID_ARG, "need nstates >= 1 and states");
    if (nstates > 0x7fffffffLL) return fail(c, QSGW_ERR_INVALID_ARG, "too many states");
    int* flags = nullptr;
    CHECK(ws_get(c, W_FLAGS, 8, &flags));
    HIP_TRY(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
    CHECK(single_begin(c, kStageSigma));
    hipLaunchKernelGGL(k_sigma_diag_self, dim3((unsigned)nstates), dim3(256), 0, c->stream, w, eps,
                       Omega, nbf, nocc, ns, eta, states, nstates, out, (int64_t)3,
                       accumulate ? 1 : 0, flags);
    CHECK(launch_check(c, "k_sigma_diag_self"));
    CHECK(single_end(c));
    int bad = 0;
    CHECK(read_flag(c, flags, &bad));
    if (bad) return fail(c, QSGW_ERR_INVALID_ARG, "a state index is outside [0, nbf)");
    return QSGW_OK;
  }
  if (mode != QSGW_SIGMA_DIAG_GRID) return fail(c, QSGW_ERR_INVALID_ARG, "unknown mode %d", mode);
  if (nomega < 1 || nstates < 1 || !omega || !states)
    return fail(c, QSGW_ERR_INVALID_ARG, "diagonal grid needs nomega, nstates >= 1");
  if (nstates > 0x7fffffffLL || (nomega + 7) / 8 > 65535)
    return fail(c, QSGW_ERR_INVALID_ARG, "grid too large");
  int* flags = nullptr;
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  HIP_TRY(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
  CHECK(single_begin(c, kStageSigma));
  hipLaunchKernelGGL(k_sigma_diag_grid, dim3((unsigned)nstates, (unsigned)((nomega + 7) / 8)),
                     dim3(256), 0, c->stream, w, eps, Omega, nbf, nocc, ns, eta, omega, nomega,
                     states, nstates, out, accumulate ? 1 : 0, flags);
  CHECK(launch_check(c, "k_sigma_diag_grid"));
  CHECK(single_end(c));
  int bad = 0;
  CHECK(read_flag(c, flags, &bad));
  if (bad) return fail(c, QSGW_ERR_INVALID_ARG, "a state index is outside [0, nbf)");
  return QSGW_OK;
}

int qsgw_hf_core(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_ao,
                 const double* C0, const double* eps0, double* h) {
  CHECK(check_common(c, nbf, naux));
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  if (!B_ao || !C0 || !eps0 || !h) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  CHECK(check_finite(c, "qsgw_hf_core", {fin(B_ao, naux * nbf * nbf, "B_ao"), fin(C0, nbf * nbf, "C0"),
                                         fin(eps0, nbf, "eps0")}));
  const int64_t nn = nbf * nbf;
  double *T = nullptr, *Bmo = nullptr, *X = nullptr, *tmp = nullptr, *tmp2 = nullptr;
  CHECK(ws_get(c, W_T, (size_t)(naux * nn), &T));
  CHECK(ws_get(c, W_BMO, (size_t)(naux * nn), &Bmo));
  CHECK(ws_get(c, W_TMP, (size_t)nn, &X));
  CHECK(ws_get(c, W_TMP2, (size_t)nn, &tmp));
  CHECK(ws_get(c, W_HMO, (size_t)nn, &tmp2));
  CHECK(stage_mo_transform(c, nbf, naux, B_ao, C0, T, Bmo));
  double *J = nullptr, *Kpart = nullptr;
  int64_t nz = 0;
  CHECK(stage_jk_mo(c, nbf, naux, nocc, Bmo, &J, &Kpart, &nz));
  hipLaunchKernelGGL(k_hf_core_mo, dim3(blocks_for(nn)), dim3(256), 0, c->stream, eps0, J, Kpart,
                     nz, nbf, X);
  CHECK(launch_check(c, "k_hf_core_mo"));
  CHECK(congruence(c, nbf, C0, X, tmp, tmp2));
  hipLaunchKernelGGL(k_symmetrize, dim3(blocks_for(nn)), dim3(256), 0, c->stream, tmp2, nbf, h);
  return launch_check(c, "k_symmetrize");
}

}  // extern "C"

namespace {

int iterate_impl(qsgw_ctx* c, const qsgw_problem* p, qsgw_state* st, const qsgw_options* o,
                 qsgw_report* rep) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (!p || !st || !o) return fail(c, QSGW_ERR_INVALID_ARG, "null argument struct");
  const int64_t nbf = p->nbf, naux = p->naux, nocc = p->nocc;
  CHECK(check_common(c, nbf, naux));
  CHECK(check_prec(c, o->precision));
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  if (!p->B_ao || !p->h || !st->eps || !st->C)
    return fail(c, QSGW_ERR_INVALID_ARG, "null problem/state pointer");
  if (!(o->eta > 0.0) || !isfinite(o->eta)) return fail(c, QSGW_ERR_INVALID_ARG, "need eta > 0");
  if (o->max_iter < 1) return fail(c, QSGW_ERR_INVALID_ARG, "need max_iter >= 1");
  if (!(o->mix > 0.0 && o->mix <= 1.0)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < mix <= 1");
  if (o->mix != 1.0 && !st->Vc)
    return fail(c, QSGW_ERR_INVALID_ARG, "mixing needs a Vc buffer in the state");
  if (o->fock_mode != QSGW_FOCK_FULL_JK && o->fock_mode != QSGW_FOCK_FROZEN)
    return fail(c, QSGW_ERR_INVALID_ARG, "unknown fock_mode %d", o->fock_mode);
  const bool frozen = o->fock_mode == QSGW_FOCK_FROZEN;
  if (o->diis != 0 && (o->diis < 2 || o->diis > 16))
    return fail(c, QSGW_ERR_INVALID_ARG, "diis must be 0 or in [2, 16]");
  if (o->diis != 0 && o->mix != 1.0)
    return fail(c, QSGW_ERR_INVALID_ARG, "diis needs mix 1");
  if (o->s_block < 0) return fail(c, QSGW_ERR_INVALID_ARG, "need s_block >= 0");
  if (!(o->near_pole >= 0.0) || !isfinite(o->near_pole))
    return fail(c, QSGW_ERR_INVALID_ARG, "need a finite near_pole >= 0");
  const bool qsmp2 = (o->flags & QSGW_OPT_QSMP2) != 0;
  if (qsmp2 && o->precision != QSGW_PREC_FP64)
    return fail(c, QSGW_ERR_UNSUPPORTED, "QSGW_OPT_QSMP2 runs in FP64 only");
  if (qsmp2 && st->diag)
    return fail(c, QSGW_ERR_UNSUPPORTED, "QSGW_OPT_QSMP2 writes no diagonal self-energy");
  const bool replay = (o->flags & QSGW_OPT_REPLAY_EIG) != 0;
  if (replay && qsmp2)
    return fail(c, QSGW_ERR_UNSUPPORTED, "QSGW_OPT_REPLAY_EIG does not apply to qsMP2 iterations");
  const bool fp32 = o->precision != QSGW_PREC_FP64;  // FP32 or split-BF16 products
  const double near = o->near_pole > 0.0 ? o->near_pole : kNearPoleDefault;

  const int64_t nv = nbf - nocc, ntr = nocc * nv, nn = nbf * nbf;
  int64_t sb = o->s_block;
  if (sb == 0) {
    // stream residues in blocks of at most ~8 GiB of w
    const int64_t cap = (int64_t)((8ull << 30) / (sizeof(double) * (uint64_t)nn));
    // (two block buffers, w and the pole-weighted copy)
    sb = ntr < cap ? ntr : (cap < 64 ? 64 : cap);
  }
  if (sb > ntr) sb = ntr;

  double *T, *Bmo, *V, *hmo, *F, *tmp, *tmp2, *epsn, *Cn, *scal;
  double *Bt = nullptr, *delta = nullptr, *sqd = nullptr, *M = nullptr, *Omega = nullptr,
         *rho = nullptr, *w = nullptr;
  int* flags;
  CHECK(ws_get(c, W_T, (size_t)(naux * nn), &T));
  CHECK(ws_get(c, W_BMO, (size_t)(naux * nn), &Bmo));
  if (!qsmp2) {
    CHECK(ws_get(c, W_BT, (size_t)(naux * ntr), &Bt));
    CHECK(ws_get(c, W_DELTA, (size_t)ntr, &delta));
    CHECK(ws_get(c, W_SQD, (size_t)ntr, &sqd));
  }
  double *M2 = nullptr, *wh = nullptr, *rhoF = nullptr, *PX = nullptr;
  float* rhoF32 = nullptr;
  unsigned long long* fprint = nullptr;
  // the two-stage solver hands the residues rho' of every excitation
  // directly (projection), the rocSOLVER path the eigenvectors Z
  const bool fold = !qsmp2 && eig_two_stage_for(c, ntr);
  if (!qsmp2) {  // (the qsMP2 potential replaces Casida, residues and the qsGW product)
    if (replay && (c->eig_ntr != ntr || c->eig_fold != fold))
      return fail(c, QSGW_ERR_INVALID_ARG,
                  "QSGW_OPT_REPLAY_EIG: the context keeps no Casida solution of %lld transitions "
                  "from the current eigensolver",
                  (long long)ntr);
    CHECK(ws_get(c, W_M, (size_t)(ntr * ntr), &M));
    CHECK(ws_get(c, W_OMEGA, (size_t)ntr, &Omega));
    if (replay) CHECK(ws_get(c, W_M2, (size_t)(ntr * ntr), &M2));
    if (fold) {
      CHECK(ws_get(c, W_RHOFULL, (size_t)(naux * ntr), &rhoF));
      if (!replay) CHECK(ws_get(c, W_EIG_PX, (size_t)(naux * ntr), &PX));
      if (o->precision == QSGW_PREC_FP32)
        CHECK(ws_get(c, W_RHOFULL32, (size_t)(naux * ntr), &rhoF32));
    }
    CHECK(ws_get(c, W_FPRINT, 2, &fprint));
    CHECK(ws_get(c, W_RHO, (size_t)(naux * sb), &rho));
    CHECK(ws_get(c, W_W, (size_t)(nn * sb), &w));
    CHECK(ws_get(c, W_WH, (size_t)(nn * sb), &wh));
  }
  CHECK(ws_get(c, W_V, (size_t)nn, &V));
  CHECK(ws_get(c, W_HMO, (size_t)nn, &hmo));
  CHECK(ws_get(c, W_F, (size_t)nn, &F));
  CHECK(ws_get(c, W_TMP, (size_t)nn, &tmp));
  CHECK(ws_get(c, W_TMP2, (size_t)nn, &tmp2));
  CHECK(ws_get(c, W_EPSN, (size_t)nbf, &epsn));
  CHECK(ws_get(c, W_CNEW, (size_t)nn, &Cn));
  CHECK(ws_get(c, W_SCAL, 8, &scal));
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  const int64_t dm = o->diis;
  double *dF = nullptr, *dE = nullptr, *dB = nullptr, *dX = nullptr;
  int* dS = nullptr;
  if (dm) {
    CHECK(ws_get(c, W_DIIS_F, (size_t)(dm * nn), &dF));
    CHECK(ws_get(c, W_DIIS_E, (size_t)(dm * nn), &dE));
    CHECK(ws_get(c, W_DIIS_B, (size_t)(16 * 16), &dB));
    CHECK(ws_get(c, W_DIIS_X, (size_t)(nn > 32 ? nn : 32), &dX));
    CHECK(ws_get(c, W_DIIS_S, (size_t)16, &dS));
    if (st->iteration == 0 || c->diis_nbf != nbf || c->diis_m != dm) {
      c->diis_n = 0;
      c->diis_next = 0;
      c->diis_nbf = nbf;
      c->diis_m = dm;
    }
  }
  float* Bmo32 = nullptr;
  if (o->precision == QSGW_PREC_FP32 && !qsmp2) {  // (the split-BF16 residue product reads split copies)
    CHECK(ws_get(c, W_BMO32, (size_t)(naux * nn), &Bmo32));
    float* r32 = nullptr;
    CHECK(ws_get(c, W_RHO32, (size_t)(naux * sb), &r32));
  }
  // The partial-sum slot is sized by its largest user before any pointer into it is taken.
  {
    double* part = nullptr;
    int64_t nz = exchange_split(c->tiles, nbf, naux, nocc).nz;
    if (qsmp2) {
      const int64_t z = mp2_split(c->tiles, nbf, mp2_block(nbf, nocc, 0) * nv).nz;
      nz = z > nz ? z : nz;
    }
    for (int64_t s0 = 0; s0 < (qsmp2 ? 0 : ntr); s0 += sb) {
      const int64_t z = sigma_slices(c->tiles, nbf, (ntr - s0) < sb ? (ntr - s0) : sb, fp32,
                                     o->precision == QSGW_PREC_SPLIT_BF16);
      nz = z > nz ? z : nz;
    }
    CHECK(ws_get(c, W_PART, (size_t)(nz * nn), &part));
    if (o->precision == QSGW_PREC_SPLIT_BF16 && !qsmp2) {
      uint16_t* u = nullptr;  // the qsGW product's split operands, sized for the largest block
      CHECK(ws_get(c, W_SPLIT_W, (size_t)(4 * x3_kfar(nbf, sb) * ((nbf + 127) / 128 * 128)), &u));
    }
    double* dummy = nullptr;
    CHECK(ws_get(c, W_J, (size_t)nn, &dummy));
    CHECK(ws_get(c, W_CP, (size_t)naux, &dummy));
    CHECK(ws_get(c, W_EIGE, (size_t)(!qsmp2 && ntr > nbf ? ntr : nbf), &dummy));
  }

  // Finite inputs (one pass over each input array).
  CHECK(check_finite(c, "qsgw_iterate",
                     {fin(p->B_ao, naux * nn, "B_ao"), fin(p->h, nn, "h"), fin(st->C, nn, "C"),
                      fin(st->eps, nbf, "eps"),
                      fin(o->mix != 1.0 && st->iteration > 0 ? st->Vc : nullptr, nn, "Vc"),
                      fin32(o->warm_start, nbf, "warm_start")}));
  HIP_TRY(c, hipMemsetAsync(flags, 0, 8 * sizeof(int), c->stream));
  if (o->warm_start) {
    // the learned warm start replaces the state's orbitals before the first iteration
    HIP_TRY(c, hipMemcpyAsync(epsn, st->eps, nbf * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(Cn, st->C, nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    CHECK(qsgw_warm_start(c, nbf, epsn, Cn, o->warm_start, st->eps, st->C));
  }

  qsgw_report local;
  memset(&local, 0, sizeof(local));
  {
    const double b = (double)nbf, a = (double)naux, t = (double)ntr, oc = (double)nocc;
    local.hot_flops = (3.0 * b + 1.0) * b * b * a    // Eq. (16): T = B C, upper triangle of C^T T
                      + t * (t + 1.0) * a            // Casida build (symmetric)
                      + (fold ? 0.0 : 2.0 * a * t * t)  // rho' (inside the eigensolve when projected)
                      + b * (b + 1.0) * a * t        // residues (symmetric in m, k)
                      + 2.0 * b * b * b * t          // qsGW matrix
                      + (frozen ? 0.0 : b * (b + 1.0) * a * oc  // exchange (symmetric)
                                          + 2.0 * a * b * b)         // Hartree
                      + 8.0 * b * b * b;             // C^T h C, C V C^T, C U
  }
  if (qsmp2) {  // the qsMP2 potential replaces Casida, residues and the qsGW product
    const double b = (double)nbf, a = (double)naux, t = (double)ntr, oc = (double)nocc;
    local.hot_flops = (3.0 * b + 1.0) * b * b * a + b * (b + 1.0) * t * a + 2.0 * b * b * b * t +
                      (frozen ? 0.0 : b * (b + 1.0) * a * oc + 2.0 * a * b * b) + 8.0 * b * b * b;
  }
  {
    const double b = (double)nbf, a = (double)naux, t = (double)ntr, oc = (double)nocc;
    local.kernel_flops[kKMo1 - kKernelBase] = 2.0 * b * b * b * a;
    local.kernel_flops[kKMo2 - kKernelBase] = b * (b + 1.0) * b * a;  // symmetric output
    local.kernel_flops[kKCasida - kKernelBase] = t * (t + 1.0) * a;
    local.kernel_flops[kKRho - kKernelBase] = fold ? 0.0 : 2.0 * a * t * t;
    local.kernel_flops[kKW - kKernelBase] = b * (b + 1.0) * a * t;
    local.kernel_flops[kKSigma - kKernelBase] = 2.0 * b * b * b * t;
    local.kernel_flops[kKSigmaRed - kKernelBase] = 0.0;
    local.kernel_flops[kKFock - kKernelBase] =
        (frozen ? 0.0 : b * (b + 1.0) * a * oc + 2.0 * a * b * b) + 8.0 * b * b * b;
  }
  int status = QSGW_NOT_CONVERGED;
  for (int64_t it = 0; it < o->max_iter; ++it) {
    const double* eps = st->eps;
    const double* C = st->C;
    Spans sp;
    sp.c = c;
    CHECK(sp.open(kStageMo));
    CHECK(stage_mo_transform(c, nbf, naux, p->B_ao, C, T, Bmo, &sp, o->precision, Bmo32));
    CHECK(sp.close());
    if (qsmp2) {
      CHECK(sp.open(kStageSigma));
      CHECK(qsgw_mp2_stage(c, nbf, naux, nocc, Bmo, eps, o->eta, V, 0, 0));
      CHECK(sp.close());
    } else {
      HIP_TRY(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
      // a replayed iteration builds its Casida matrix apart and keeps the solved eigenpairs
      double* Mb = replay ? M2 : M;
      if (!replay) c->eig_ntr = -1;  // W_M is about to be overwritten
      CHECK(sp.open(kStageRpa));
      CHECK(stage_rpa_build(c, nbf, naux, nocc, Bmo, eps, Mb, sqd, delta, Bt, flags, &sp,
                            o->precision));
      CHECK(sp.close());
      // bit fingerprint of the matrix (outside the timed stages)
      HIP_TRY(c, hipMemsetAsync(fprint, 0, sizeof(unsigned long long), c->stream));
      hipLaunchKernelGGL(k_bits_fingerprint, dim3(2048), dim3(256), 0, c->stream, Mb, ntr * ntr,
                         fprint);
      CHECK(launch_check(c, "k_bits_fingerprint"));
      unsigned long long fp = 0;
      HIP_TRY(c, hipMemcpyAsync(&fp, fprint, sizeof(fp), hipMemcpyDeviceToHost, c->stream));
      {
        int bad = 0;
        CHECK(read_flag(c, flags, &bad));  // (synchronizes: fp is read too)
        if (bad) return fail(c, QSGW_ERR_INVALID_ARG, "orbital energies are not in aufbau order");
      }
      if (replay) {
        if (fp != c->eig_fp)
          return fail(c, QSGW_ERR_INVALID_ARG,
                      "QSGW_OPT_REPLAY_EIG: the Casida matrix differs from the one last solved");
      } else {
        CHECK(sp.open(kStageEigRpa));
        if (fold)
          CHECK(stage_rpa_solve_project(c, ntr, naux, M, Omega, Bt, PX, rhoF));
        else
          CHECK(stage_rpa_solve(c, ntr, M, Omega));
        CHECK(sp.close());
        c->eig_ntr = ntr;
        c->eig_fp = fp;
        c->eig_fold = fold;
      }
      if (fold && rhoF32) {
        hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(naux * ntr)), dim3(256), 0, c->stream, rhoF,
                           naux * ntr, rhoF32);
        CHECK(launch_check(c, "k_to_f32"));
      }
      for (int64_t s0 = 0; s0 < ntr; s0 += sb) {
        const int64_t ns = (ntr - s0) < sb ? (ntr - s0) : sb;
        CHECK(sp.open(kStageRes));
        if (fp32) {
          // FP32 products: the pole-weighted copy and w in FP32 share the wh buffer
          // (the FP64 residues are written only for the diagonal outputs)
          float* wh32 = reinterpret_cast<float*>(wh);
          float* w32 = wh32 + nn * ns;
          double* w64 = (it == 0 && st->diag) ? w : nullptr;
          // split-BF16: the residue epilogue also writes the qsGW product's split operands
          X3Out x3o{};
          const bool x3 = o->precision == QSGW_PREC_SPLIT_BF16;
          if (x3) {
            x3o.cs = (nbf + 127) / 128 * 128;
            x3o.nsp = (ns + 7) / 8 * 8;
            x3o.kfar = x3_kfar(nbf, ns);
            x3o.ws = static_cast<uint16_t*>(c->ws[W_SPLIT_W].p);
            x3o.whs = x3o.ws + 2 * x3o.plane();
            // the near-pole terms first: the residue epilogue keeps FP32
            // residues only in the columns the near-pole part reads
            CHECK(near_x3(c, nbf, nocc, ns, eps, Omega + s0, near, &x3o));
          }
          CHECK(stage_residues(c, nbf, naux, ntr, Bmo, Bt, M, Omega, s0, ns,
                               fold ? rhoF + s0 : rho, w64, &sp, nullptr, eps, nocc, o->eta,
                               o->precision, wh32, w32, near, Bmo32,
                               static_cast<const float*>(c->ws[W_BT32].p), s0 > 0,
                               x3 ? &x3o : nullptr, fold, fold ? ntr : 0,
                               rhoF32 ? rhoF32 + s0 : nullptr));
          CHECK(sp.close());
          CHECK(sp.open(kStageSigma));
          if (x3)
            CHECK(stage_sigma_qs32_t<Bf16x3>(c, nbf, nocc, ns, wh32, w32, eps, Omega + s0, o->eta,
                                             near, V, s0 > 0 ? 1 : 0, &sp, &x3o));
          else
            CHECK(stage_sigma_qs32_t<float>(c, nbf, nocc, ns, wh32, w32, eps, Omega + s0, o->eta,
                                            near, V, s0 > 0 ? 1 : 0, &sp));
        } else {
          CHECK(stage_residues(c, nbf, naux, ntr, Bmo, Bt, M, Omega, s0, ns,
                               fold ? rhoF + s0 : rho, w, &sp, wh, eps, nocc, o->eta,
                               o->precision, nullptr, nullptr, 0.0, nullptr, nullptr, false,
                               nullptr, fold, fold ? ntr : 0));
          CHECK(sp.close());
          CHECK(sp.open(kStageSigma));
          CHECK(stage_sigma_qs(c, nbf, nocc, ns, w, eps, Omega + s0, o->eta, V, s0 > 0 ? 1 : 0, &sp,
                               wh));
        }
        CHECK(sp.close());
        if (it == 0 && st->diag) {
          hipLaunchKernelGGL(k_sigma_diag_self, dim3((unsigned)nbf), dim3(256), 0, c->stream, w, eps,
                             Omega + s0, nbf, nocc, ns, o->eta, (const int64_t*)nullptr, nbf,
                             st->diag, (int64_t)4, s0 > 0 ? 1 : 0, flags + 3);
          CHECK(launch_check(c, "k_sigma_diag_self"));
        }
      }
      if (it == 0 && st->diag) {
        hipLaunchKernelGGL(k_exchange_diag, dim3((unsigned)nbf), dim3(256), 0, c->stream, Bmo, naux,
                           nbf, nocc, st->diag + 3, (int64_t)4);
        CHECK(launch_check(c, "k_exchange_diag"));
      }
    }
    CHECK(sp.open(kStageFock));
    CHECK(sp.open(kKFock));
    // correlation potential in the AO basis (output and mixing)
    if (st->Vc) {
      CHECK(congruence(c, nbf, C, V, tmp, tmp2));
      if (o->mix != 1.0 && st->iteration > 0) {
        hipLaunchKernelGGL(k_axpby, dim3(blocks_for(nn)), dim3(256), 0, c->stream, tmp2, st->Vc,
                           o->mix, 1.0 - o->mix, nn, tmp2);
        CHECK(launch_check(c, "k_axpby"));
        hipLaunchKernelGGL(k_symmetrize, dim3(blocks_for(nn)), dim3(256), 0, c->stream, tmp2, nbf,
                           st->Vc);
        CHECK(launch_check(c, "k_symmetrize"));
        // back to the MO basis of the current orbitals for the Fock build
        CHECK(congruence_t(c, nbf, C, st->Vc, tmp, tmp2));
        hipLaunchKernelGGL(k_symmetrize, dim3(blocks_for(nn)), dim3(256), 0, c->stream, tmp2, nbf,
                           V);
        CHECK(launch_check(c, "k_symmetrize"));
      } else {
        hipLaunchKernelGGL(k_symmetrize, dim3(blocks_for(nn)), dim3(256), 0, c->stream, tmp2, nbf,
                           st->Vc);
        CHECK(launch_check(c, "k_symmetrize"));
      }
    }
    // Eq. (6) in the MO basis of the current orbitals: C^T h C + J - K + V
    // (frozen mean field: C^T h C + V)
    CHECK(congruence_t(c, nbf, C, p->h, tmp, hmo));
    if (frozen) {
      hipLaunchKernelGGL(k_fock_frozen, dim3(blocks_for(nn)), dim3(256), 0, c->stream, hmo, V, nbf,
                         F);
      CHECK(launch_check(c, "k_fock_frozen"));
    } else {
      double *J = nullptr, *Kpart = nullptr;
      int64_t nz = 0;
      CHECK(stage_jk_mo(c, nbf, naux, nocc, Bmo, &J, &Kpart, &nz));
      hipLaunchKernelGGL(k_fock_assemble, dim3(blocks_for(nn)), dim3(256), 0, c->stream, hmo, J,
                         Kpart, nz, V, nbf, F);
      CHECK(launch_check(c, "k_fock_assemble"));
    }
    if (dm) {
      // Pulay DIIS: keep F (AO basis) and its commutator error, then
      // diagonalise the combination of the kept Fock matrices with the
      // weights that minimise the combined error (first iteration: F itself)
      const int64_t k = c->diis_next;
      CHECK(congruence(c, nbf, C, F, tmp, dF + k * nn));
      hipLaunchKernelGGL(k_diis_error_mo, dim3(blocks_for(nn)), dim3(256), 0, c->stream, F, nbf,
                         nocc, tmp2);
      CHECK(launch_check(c, "k_diis_error_mo"));
      CHECK(congruence(c, nbf, C, tmp2, tmp, dE + k * nn));
      const int64_t na = c->diis_n < dm ? c->diis_n + 1 : dm;
      for (int64_t i = 0; i < na; ++i) c->diis_slots[i] = (int)((k - (na - 1) + i + dm) % dm);
      HIP_TRY(c, hipMemcpyAsync(dS, c->diis_slots, na * sizeof(int), hipMemcpyHostToDevice,
                                c->stream));
      hipLaunchKernelGGL(k_diis_dots, dim3((unsigned)na), dim3(256), 0, c->stream, dE, nn, k, dS,
                         dB, (int64_t)16);
      CHECK(launch_check(c, "k_diis_dots"));
      if (na > 1) {
        hipLaunchKernelGGL(k_diis_solve, dim3(1), dim3(64), 0, c->stream, dB, (int64_t)16, dS,
                           (int)na, dX, flags + 6);
        hipLaunchKernelGGL(k_diis_combine, dim3(blocks_for(nn)), dim3(256), 0, c->stream, dF, nn,
                           dS, (int)na, dX, tmp2);
        CHECK(launch_check(c, "k_diis_combine"));
        // back to the MO basis of the current orbitals
        CHECK(congruence_t(c, nbf, C, tmp2, tmp, dX));
        hipLaunchKernelGGL(k_symmetrize, dim3(blocks_for(nn)), dim3(256), 0, c->stream, dX, nbf, F);
        CHECK(launch_check(c, "k_symmetrize"));
      }
      c->diis_n = na;
      c->diis_next = (k + 1) % dm;
    }
    CHECK(sp.close());
    CHECK(sp.close());
    CHECK(sp.open(kStageEigFock));
    CHECK(syevd(c, nbf, F, epsn, "eig_fock"));
    CHECK(sp.close());
    // C' = C U (U column-major in F), sign convention, max |d eps|
    {
      Strided<true> A{C, nbf, 1, 0, nbf};
      Strided<true> B{F, nbf, 1, 0, nbf};
      EpiStore E{Cn, nbf, 0, 0, 1.0};
      CHECK((gemm<64, 64, false>(c, "rotate_orbitals", A, B, E, nbf, nbf, nbf, 1)));
    }
    hipLaunchKernelGGL(k_fix_column_signs, dim3((unsigned)nbf), dim3(256), 0, c->stream, Cn, nbf);
    hipLaunchKernelGGL(k_max_abs_diff, dim3(1), dim3(256), 0, c->stream, epsn, st->eps, nbf, scal);
    CHECK(launch_check(c, "k_max_abs_diff"));
    HIP_TRY(c, hipMemcpyAsync(st->eps, epsn, nbf * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(st->C, Cn, nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    double dmax = 0.0;
    HIP_TRY(c, hipMemcpyAsync(&dmax, scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));

    for (const auto& span : sp.v) {
      const double ms = elapsed(c, span.e0, span.e1);
      if (span.id >= kKernelBase) {
        local.ms_kernel[span.id - kKernelBase] += ms;
        local.kernel_launches[span.id - kKernelBase] += 1;
      } else {
        local.ms_stage[span.id] += ms;
      }
    }

    if (local.iterations < QSGW_REPORT_MAX_ITERS) local.max_deps[local.iterations] = dmax;
    local.iterations++;
    st->iteration++;
    if (!isfinite(dmax)) {
      if (rep) *rep = local;
      return fail(c, QSGW_ERR_NONFINITE, "non-finite orbital energies after iteration %lld",
                  (long long)st->iteration);
    }
    if (dmax < o->tol) {
      status = QSGW_OK;
      local.converged = 1;
      break;
    }
  }
  for (int i = 0; i < 7; ++i) c->stage_ms[i] = local.ms_stage[i];
  c->last_stage = -1;
  if (rep) *rep = local;
  return status;
}

}  // namespace

extern "C" {

int qsgw_iterate(qsgw_ctx* c, const qsgw_problem* p, qsgw_state* st, const qsgw_options* o,
                 qsgw_report* rep) {
  const bool refine = o && (o->flags & QSGW_OPT_REFINE) && o->precision != QSGW_PREC_FP64;
  if (!refine) return iterate_impl(c, p, st, o, rep);
  // reduced-precision iterations, then one FP64 iteration from where they stopped
  qsgw_report r1, r2;
  memset(&r1, 0, sizeof(r1));
  memset(&r2, 0, sizeof(r2));
  const int rc1 = iterate_impl(c, p, st, o, &r1);
  if (rc1 < 0) {
    if (rep) *rep = r1;
    return rc1;
  }
  qsgw_options o2 = *o;
  o2.precision = QSGW_PREC_FP64;
  o2.max_iter = 1;
  o2.flags &= ~(int64_t)QSGW_OPT_REFINE;
  double* diag = st->diag;  // diagonal outputs belong to the call's first iteration
  st->diag = nullptr;
  const int rc2 = iterate_impl(c, p, st, &o2, &r2);
  st->diag = diag;
  if (rep) {
    qsgw_report r = r1;
    if (r.iterations < QSGW_REPORT_MAX_ITERS) r.max_deps[r.iterations] = r2.max_deps[0];
    r.iterations += r2.iterations;
    r.converged = r2.converged;
    for (int k = 0; k < 7; ++k) r.ms_stage[k] += r2.ms_stage[k];
    for (int k = 0; k < 8; ++k) {
      r.ms_kernel[k] += r2.ms_kernel[k];
      r.kernel_launches[k] += r2.kernel_launches[k];
    }
    *rep = r;
  }
  return rc2;
}

// Open-shell GW potential, FP64.  Transitions of both spins share one Casida
// problem (spin alpha first); the concatenated Bt carries sqrt(Delta) / sqrt(2),
// so the closed-shell kernels give the open-shell factors: the Casida epilogue's
// 4 Bt^T Bt becomes 2 K sqrt(Delta)..sqrt(Delta), and rho' = sqrt(2 / Omega) Bt Z^T
// becomes the spin-resolved sqrt(1 / Omega) B_ia (X+Y) sum without the singlet sqrt(2).
int qsgw_gw_unrestricted(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc_a, int64_t nocc_b,
                         const double* B_mo_a, const double* B_mo_b, const double* eps_a,
                         const double* eps_b, double eta, double* V_a, double* V_b,
                         double* Omega_out, int precision) {
  CHECK(check_common(c, nbf, naux));
  if (!(nocc_a > 0 && nocc_a < nbf && nocc_b > 0 && nocc_b < nbf))
    return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc_a, nocc_b < nbf");
  if (!(eta > 0.0) || !isfinite(eta)) return fail(c, QSGW_ERR_INVALID_ARG, "need finite eta > 0");
  if (!B_mo_a || !B_mo_b || !eps_a || !eps_b || !V_a || !V_b)
    return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  if (precision != QSGW_PREC_FP64)
    return fail(c, QSGW_ERR_UNSUPPORTED, "qsgw_gw_unrestricted: FP64 only (precision %d)", precision);
  CHECK(check_finite(c, "qsgw_gw_unrestricted",
                     {fin(B_mo_a, naux * nbf * nbf, "B_mo_a"), fin(B_mo_b, naux * nbf * nbf, "B_mo_b"),
                      fin(eps_a, nbf, "eps_a"), fin(eps_b, nbf, "eps_b")}));
  const int64_t nn = nbf * nbf;
  const int64_t no[2] = {nocc_a, nocc_b};
  const int64_t nt[2] = {nocc_a * (nbf - nocc_a), nocc_b * (nbf - nocc_b)};
  const int64_t ntr = nt[0] + nt[1];
  const double* Bs[2] = {B_mo_a, B_mo_b};
  const double* es[2] = {eps_a, eps_b};
  double* Vs[2] = {V_a, V_b};
  if (ntr > 46340) return fail(c, QSGW_ERR_INVALID_ARG, "too many transitions for one Casida matrix");
  c->eig_ntr = -1;  // W_M and W_OMEGA are reused here
  double *Bt, *delta, *sqd, *M, *Omega, *rho, *w, *wh;
  int* flags;
  CHECK(ws_get(c, W_BT, (size_t)(naux * ntr), &Bt));
  CHECK(ws_get(c, W_DELTA, (size_t)ntr, &delta));
  CHECK(ws_get(c, W_SQD, (size_t)ntr, &sqd));
  CHECK(ws_get(c, W_M, (size_t)(ntr * ntr), &M));
  CHECK(ws_get(c, W_OMEGA, (size_t)ntr, &Omega));
  CHECK(ws_get(c, W_FLAGS, 8, &flags));
  const int64_t cap = (int64_t)((8ull << 30) / (sizeof(double) * (uint64_t)nn));
  const int64_t sb = ntr < cap ? ntr : (cap < 64 ? 64 : cap);
  CHECK(ws_get(c, W_RHO, (size_t)(naux * sb), &rho));
  CHECK(ws_get(c, W_W, (size_t)(nn * sb), &w));
  CHECK(ws_get(c, W_WH, (size_t)(nn * sb), &wh));
  // with the two-stage solver the eigensolve hands rho' of every excitation
  // (projection of the spin-stacked Bt, the eigenvectors never formed)
  const bool fold = eig_two_stage_for(c, ntr);
  double *PX = nullptr, *rhoF = nullptr;
  if (fold) {
    CHECK(ws_get(c, W_EIG_PX, (size_t)(naux * ntr), &PX));
    CHECK(ws_get(c, W_RHOFULL, (size_t)(naux * ntr), &rhoF));
  }
  Spans spn;
  spn.c = c;
  HIP_TRY(c, hipMemsetAsync(flags, 0, sizeof(int), c->stream));
  CHECK(spn.open(kStageRpa));
  int64_t off = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t nv = nbf - no[sp];
    hipLaunchKernelGGL(k_transitions, dim3(blocks_for(nt[sp])), dim3(256), 0, c->stream, es[sp],
                       no[sp], nv, delta + off, sqd + off, flags);
    CHECK(launch_check(c, "k_transitions"));
    hipLaunchKernelGGL(k_gather_bia_ld, dim3(blocks_for(naux * nt[sp])), dim3(256), 0, c->stream,
                       Bs[sp], sqd + off, 1.0 / sqrt(2.0), naux, nbf, no[sp], ntr, Bt + off);
    CHECK(launch_check(c, "k_gather_bia_ld"));
    off += nt[sp];
  }
  int bad = 0;
  CHECK(read_flag(c, flags, &bad));
  if (bad) return fail(c, QSGW_ERR_INVALID_ARG, "need eps[a] > eps[i] for every transition");
  {
    EpiCasida E{M, delta, ntr};
    Strided<false> A{Bt, 1, ntr, 0, ntr};
    CHECK((gemm_shape<double, true>(c, c->tiles.shape[TU_CASIDA], "gw_unrestricted/casida", A, A,
                                    E, ntr, ntr, naux, 1)));
  }
  CHECK(spn.close());
  CHECK(spn.open(kStageEigRpa));
  if (fold)
    CHECK(stage_rpa_solve_project(c, ntr, naux, M, Omega, Bt, PX, rhoF));
  else
    CHECK(stage_rpa_solve(c, ntr, M, Omega));
  CHECK(spn.close());
  for (int64_t s0 = 0; s0 < ntr; s0 += sb) {
    const int64_t ns = ntr - s0 < sb ? ntr - s0 : sb;
    for (int sp = 0; sp < 2; ++sp) {
      // rho' of the block is shared by both spins (from the projection, or made by the first)
      CHECK(spn.open(kStageRes));
      CHECK(stage_residues(c, nbf, naux, ntr, Bs[sp], Bt, M, Omega, s0, ns,
                           fold ? rhoF + s0 : rho, w, nullptr, wh, es[sp], no[sp], eta,
                           QSGW_PREC_FP64, nullptr, nullptr, 0.0, nullptr, nullptr, false, nullptr,
                           fold || sp > 0, fold ? ntr : 0));
      CHECK(spn.close());
      CHECK(spn.open(kStageSigma));
      CHECK(stage_sigma_qs(c, nbf, no[sp], ns, w, es[sp], Omega + s0, eta, Vs[sp],
                           s0 > 0 ? 1 : 0, nullptr, wh));
      CHECK(spn.close());
    }
  }
  if (Omega_out)
    HIP_TRY(c, hipMemcpyAsync(Omega_out, Omega, (size_t)ntr * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < 7; ++i) c->stage_ms[i] = 0.0;
  for (const auto& span : spn.v) c->stage_ms[span.id] += elapsed(c, span.e0, span.e1);
  c->last_stage = -1;  // qsgw_last_stage_ms reports stage_ms as set here
  return QSGW_OK;
}

// Open-shell Fock update in the MO basis of each spin's current orbitals:
// F = C^T h C + J - K + V with J from both spins' densities (the Hartree kernel
// doubles its trace vector, so it gets half the summed traces) and K from that
// spin's occupied orbitals; then eigenvectors U, C' = C U, signs fixed.
int qsgw_fock_unrestricted(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc_a, int64_t nocc_b,
                           const double* B_mo_a, const double* B_mo_b, const double* h,
                           const double* V_a, const double* V_b, double* eps_a, double* eps_b,
                           double* C_a, double* C_b) {
  CHECK(check_common(c, nbf, naux));
  if (!(nocc_a > 0 && nocc_a < nbf && nocc_b > 0 && nocc_b < nbf))
    return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc_a, nocc_b < nbf");
  if (!B_mo_a || !B_mo_b || !h || !V_a || !V_b || !eps_a || !eps_b || !C_a || !C_b)
    return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  CHECK(check_finite(c, "qsgw_fock_unrestricted",
                     {fin(B_mo_a, naux * nbf * nbf, "B_mo_a"), fin(B_mo_b, naux * nbf * nbf, "B_mo_b"),
                      fin(h, nbf * nbf, "h"), fin(V_a, nbf * nbf, "V_a"), fin(V_b, nbf * nbf, "V_b"),
                      fin(C_a, nbf * nbf, "C_a"), fin(C_b, nbf * nbf, "C_b")}));
  const int64_t nn = nbf * nbf;
  const int64_t no[2] = {nocc_a, nocc_b};
  const double* Bs[2] = {B_mo_a, B_mo_b};
  const double* Vs[2] = {V_a, V_b};
  double* es[2] = {eps_a, eps_b};
  double* Cs[2] = {C_a, C_b};
  double *cp, *J, *hmo, *F, *tmp, *epsn, *Cn;
  CHECK(ws_get(c, W_CP, (size_t)(3 * naux), &cp));
  CHECK(ws_get(c, W_J, (size_t)nn, &J));
  CHECK(ws_get(c, W_HMO, (size_t)nn, &hmo));
  CHECK(ws_get(c, W_F, (size_t)nn, &F));
  CHECK(ws_get(c, W_TMP, (size_t)nn, &tmp));
  CHECK(ws_get(c, W_EPSN, (size_t)nbf, &epsn));
  CHECK(ws_get(c, W_CNEW, (size_t)nn, &Cn));
  CHECK(single_begin(c, kStageFock));
  for (int sp = 0; sp < 2; ++sp) {
    hipLaunchKernelGGL(k_occ_trace, dim3(blocks_for(naux)), dim3(256), 0, c->stream, Bs[sp], naux,
                       nbf, no[sp], cp + sp * naux);
    CHECK(launch_check(c, "k_occ_trace"));
  }
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(naux)), dim3(256), 0, c->stream, cp, cp + naux, 0.5,
                     0.5, naux, cp + 2 * naux);
  CHECK(launch_check(c, "k_axpby"));
  for (int sp = 0; sp < 2; ++sp) {
    constexpr int64_t pg = 32;
    const int64_t ng = (naux + pg - 1) / pg;
    double* jp = nullptr;
    CHECK(ws_get(c, W_REDPART, (size_t)(ng * nn), &jp));
    hipLaunchKernelGGL(k_hartree_part, dim3(blocks_for(ng * nn)), dim3(256), 0, c->stream, Bs[sp],
                       cp + 2 * naux, naux, nn, pg, jp);
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks_for(nn)), dim3(256), 0, c->stream, jp, ng, nn, ng,
                       J);
    CHECK(launch_check(c, "k_hartree_part"));
    const SplitPlan spl = exchange_split(c->tiles, nbf, naux, no[sp]);
    double* Kpart = nullptr;
    CHECK(ws_get(c, W_PART, (size_t)(spl.nz * nn), &Kpart));
    {
      OccRowsOp A{Bs[sp], nbf, no[sp]};
      EpiStore E{Kpart, nbf, 0, nn, 1.0};
      CHECK((gemm_shape<double, true>(c, c->tiles.shape[TU_EXCHANGE], "fock_u/exchange", A, A, E,
                                      nbf, nbf, naux * no[sp], 1, spl)));
    }
    CHECK(congruence_t(c, nbf, Cs[sp], h, tmp, hmo));
    hipLaunchKernelGGL(k_fock_assemble, dim3(blocks_for(nn)), dim3(256), 0, c->stream, hmo, J,
                       Kpart, spl.nz, Vs[sp], nbf, F);
    CHECK(launch_check(c, "k_fock_assemble"));
    CHECK(syevd(c, nbf, F, epsn, "fock_u/eig"));
    {  // C' = C U (U column-major in F)
      Strided<true> A{Cs[sp], nbf, 1, 0, nbf};
      Strided<true> B{F, nbf, 1, 0, nbf};
      EpiStore E{Cn, nbf, 0, 0, 1.0};
      CHECK((gemm<64, 64, false>(c, "fock_u/rotate", A, B, E, nbf, nbf, nbf, 1)));
    }
    hipLaunchKernelGGL(k_fix_column_signs, dim3((unsigned)nbf), dim3(256), 0, c->stream, Cn, nbf);
    CHECK(launch_check(c, "k_fix_column_signs"));
    HIP_TRY(c, hipMemcpyAsync(es[sp], epsn, nbf * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(Cs[sp], Cn, nn * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
  }
  return single_end(c);
}

int qsgw_iterate_unrestricted(qsgw_ctx* c, const qsgw_problem* p, int64_t nocc_b,
                              qsgw_state* st_a, qsgw_state* st_b, const qsgw_options* o,
                              qsgw_report* rep) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (!p || !st_a || !st_b || !o) return fail(c, QSGW_ERR_INVALID_ARG, "null argument struct");
  const int64_t nbf = p->nbf, naux = p->naux, na = p->nocc, nb = nocc_b, nn = nbf * nbf;
  CHECK(check_common(c, nbf, naux));
  if (!(na > 0 && na < nbf && nb > 0 && nb < nbf))
    return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc_a, nocc_b < nbf");
  if (!p->B_ao || !p->h || !st_a->eps || !st_a->C || !st_b->eps || !st_b->C)
    return fail(c, QSGW_ERR_INVALID_ARG, "null problem/state pointer");
  if (!(o->eta > 0.0) || !isfinite(o->eta)) return fail(c, QSGW_ERR_INVALID_ARG, "need eta > 0");
  if (o->max_iter < 1) return fail(c, QSGW_ERR_INVALID_ARG, "need max_iter >= 1");
  if (o->precision != QSGW_PREC_FP64 || o->mix != 1.0 || o->fock_mode != QSGW_FOCK_FULL_JK ||
      o->flags != 0 || o->s_block != 0 || o->warm_start || o->diis != 0 || st_a->Vc || st_b->Vc ||
      st_a->diag || st_b->diag)
    return fail(c, QSGW_ERR_UNSUPPORTED,
                "qsgw_iterate_unrestricted: FP64, mix 1, QSGW_FOCK_FULL_JK, no flags, automatic "
                "blocks, no warm start or DIIS and no Vc/diag outputs only");
  double *Bma, *Bmb, *Va, *Vb, *old;
  CHECK(ws_get(c, W_BMO, (size_t)(naux * nn), &Bma));
  CHECK(ws_get(c, W_BMO_B, (size_t)(naux * nn), &Bmb));
  CHECK(ws_get(c, W_V, (size_t)nn, &Va));
  CHECK(ws_get(c, W_VB, (size_t)nn, &Vb));
  CHECK(ws_get(c, W_TMP2, (size_t)(nn > 2 * nbf ? nn : 2 * nbf), &old));
  qsgw_report local;
  memset(&local, 0, sizeof(local));
  {
    const double b = (double)nbf, a = (double)naux;
    const double t = (double)(na * (nbf - na) + nb * (nbf - nb));
    local.hot_flops = 2.0 * (3.0 * b + 1.0) * b * b * a    // Eq. (16), both spins
                      + t * (t + 1.0) * a + 2.0 * a * t * t  // Casida build and rho' (shared)
                      + 2.0 * (b * (b + 1.0) * a * t + 2.0 * b * b * b * t)  // residues + Eq. (19)
                      + b * (b + 1.0) * a * (double)(na + nb) + 2.0 * a * b * b + 16.0 * b * b * b;
  }
  auto add_ms = [&](void) -> int {
    double ms[7];
    CHECK(qsgw_last_stage_ms(c, ms, 7));
    for (int i = 0; i < 7; ++i) local.ms_stage[i] += ms[i];
    return QSGW_OK;
  };
  std::vector<double> h_old((size_t)(2 * nbf)), h_new((size_t)(2 * nbf));
  int status = QSGW_NOT_CONVERGED;
  for (int64_t it = 0; it < o->max_iter; ++it) {
    CHECK(qsgw_mo_transform(c, nbf, naux, p->B_ao, st_a->C, Bma, QSGW_PREC_FP64));
    CHECK(add_ms());
    CHECK(qsgw_mo_transform(c, nbf, naux, p->B_ao, st_b->C, Bmb, QSGW_PREC_FP64));
    CHECK(add_ms());
    CHECK(qsgw_gw_unrestricted(c, nbf, naux, na, nb, Bma, Bmb, st_a->eps, st_b->eps, o->eta, Va,
                               Vb, nullptr, QSGW_PREC_FP64));
    CHECK(add_ms());
    HIP_TRY(c, hipMemcpyAsync(old, st_a->eps, nbf * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(old + nbf, st_b->eps, nbf * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    CHECK(qsgw_fock_unrestricted(c, nbf, naux, na, nb, Bma, Bmb, p->h, Va, Vb, st_a->eps,
                                 st_b->eps, st_a->C, st_b->C));
    CHECK(add_ms());
    HIP_TRY(c, hipMemcpyAsync(h_old.data(), old, 2 * nbf * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(h_new.data(), st_a->eps, nbf * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(h_new.data() + nbf, st_b->eps, nbf * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double d = 0.0;
    for (int64_t m = 0; m < 2 * nbf; ++m) d = fmax(d, fabs(h_new[(size_t)m] - h_old[(size_t)m]));
    if (it < QSGW_REPORT_MAX_ITERS) local.max_deps[it] = d;
    local.iterations = it + 1;
    ++st_a->iteration;
    ++st_b->iteration;
    if (d < o->tol) {
      status = QSGW_OK;
      local.converged = 1;
      break;
    }
  }
  if (rep) *rep = local;
  return status;
}

int qsgw_set_eigensolver(qsgw_ctx* c, int solver) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  if (solver != QSGW_EIG_AUTO && solver != QSGW_EIG_ROCSOLVER && solver != QSGW_EIG_TWO_STAGE)
    return fail(c, QSGW_ERR_INVALID_ARG, "unknown eigensolver %d", solver);
  c->eig_solver = solver;
  return QSGW_OK;
}

int qsgw_set_tiles(qsgw_ctx* c, const char* spec) {
  if (!c) return QSGW_ERR_INVALID_ARG;
  Tiles t;  // defaults
  if (spec && *spec) {
    static const char* names[TU_COUNT] = {"mo1", "mo2", "casida", "rho", "sigma", "exchange"};
    static const bool square[TU_COUNT] = {false, true, true, false, false, true};
    std::string all(spec);
    size_t pos = 0;
    while (pos <= all.size()) {
      size_t end = all.find(',', pos);
      if (end == std::string::npos) end = all.size();
      const std::string item = all.substr(pos, end - pos);
      pos = end + 1;
      if (item.empty()) continue;
      const size_t eq = item.find('=');
      if (eq == std::string::npos) return fail(c, QSGW_ERR_INVALID_ARG, "tiles: no '=' in '%s'", item.c_str());
      const std::string key = item.substr(0, eq), val = item.substr(eq + 1);
      bool done = false;
      for (int k = 0; k < TU_COUNT && !done; ++k) {
        if (key != names[k]) continue;
        int sh = -1;
        if (val == "64x64") sh = SH_64x64;
        else if (val == "128x64") sh = SH_128x64;
        else if (val == "128x128") sh = SH_128x128;
        if (sh < 0 || (square[k] && sh == SH_128x64))
          return fail(c, QSGW_ERR_INVALID_ARG, "tiles: shape '%s' not available for %s", val.c_str(),
                      key.c_str());
        t.shape[k] = sh;
        done = true;
      }
      if (done) continue;
      char* e = nullptr;
      const long long v = strtoll(val.c_str(), &e, 10);
      if (key == "persistent") {
        if (!e || *e || v < 0 || v > 8)
          return fail(c, QSGW_ERR_INVALID_ARG, "tiles: persistent needs an integer in [0, 8]");
        t.persistent = v;
        continue;
      }
      if (key == "panel_coop") {
        if (!e || *e || v < 0 || v > 1)
          return fail(c, QSGW_ERR_INVALID_ARG, "tiles: panel_coop needs 0 or 1");
        t.panel_coop = v;
        continue;
      }
      if (key == "dc_leaf") {
        if (!e || *e || v < 16 || v > 46340)
          return fail(c, QSGW_ERR_INVALID_ARG, "tiles: dc_leaf needs an integer in [16, 46340]");
        t.dc_leaf = v;
        continue;
      }
      int64_t* target = key == "sigma_target" ? &t.sigma_target
                        : key == "rho_target" ? &t.rho_target
                        : key == "exchange_target" ? &t.exchange_target
                        : key == "mp2_target"      ? &t.mp2_target
                                                    : nullptr;
      if (!target) return fail(c, QSGW_ERR_INVALID_ARG, "tiles: unknown key '%s'", key.c_str());
      if (!e || *e || v < 64 || v > (1 << 20))
        return fail(c, QSGW_ERR_INVALID_ARG, "tiles: %s needs an integer in [64, 2^20]", key.c_str());
      *target = v;
    }
  }
  // work queued with the previous table may still run; the table only affects launches
  c->tiles = t;
  return QSGW_OK;
}

int qsgw_get_tiles(qsgw_ctx* c, char* buf, int64_t size) {
  if (!c || !buf || size < 1) return QSGW_ERR_INVALID_ARG;
  static const char* names[TU_COUNT] = {"mo1", "mo2", "casida", "rho", "sigma", "exchange"};
  static const char* shapes[SH_COUNT] = {"64x64", "128x64", "128x128"};
  std::string out;
  for (int k = 0; k < TU_COUNT; ++k) {
    out += names[k];
    out += "=";
    out += shapes[c->tiles.shape[k]];
    out += ",";
  }
  out += "sigma_target=" + std::to_string(c->tiles.sigma_target);
  out += ",rho_target=" + std::to_string(c->tiles.rho_target);
  out += ",exchange_target=" + std::to_string(c->tiles.exchange_target);
  out += ",persistent=" + std::to_string(c->tiles.persistent);
  out += ",mp2_target=" + std::to_string(c->tiles.mp2_target);
  out += ",dc_leaf=" + std::to_string(c->tiles.dc_leaf);
  out += ",panel_coop=" + std::to_string(c->tiles.panel_coop);
  if ((int64_t)out.size() + 1 > size) return fail(c, QSGW_ERR_INVALID_ARG, "buffer too small");
  memcpy(buf, out.c_str(), out.size() + 1);
  return QSGW_OK;
}

}  // extern "C"
