// qsMP2 potential, Eqs. (20)-(21), closed shell, real orbitals, FP64 matrix
// cores.  With c = (p, t), t = (i, a) a transition (i occupied, a empty) and
//   D[m][c]  = (mp|ia)                                   (RI integrals)
//   Rh[n][c] = (2 (np|ia) - X_npia) Re g_c(eps_n)        (pole-weighted)
//   X = (pi|an) for empty p, (pa|in) for occupied p,
//   Re g_c(w) = x / (x^2 + eta^2), x = w - (eps_p + eps_i - eps_a) for
//   occupied p, x = w - (eps_p + eps_a - eps_i) for empty p,
// Eq. (20) gives Re Sigma_mn(eps_n) = G[m][n], G = D Rh^T, and Eq. (21)
// V = 1/2 (G + G^T).  Both exchange integrals are entries of D itself:
// (pi|an) = D[n][a][(i, p)] sits in the same block of transitions (same i),
// (pa|in) = D[n][i][(p, a)] in the block of occupied state p, so with more
// than one block the integrals (ni|pa) of every occupied i are kept apart.
#include "internal.hpp"

namespace {

int stage_mp2(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
              const double* eps, double eta, double* V, int64_t occ_block, int accumulate) {
  const int64_t nv = nbf - nocc, ntr = nocc * nv, nn = nbf * nbf;
  const int64_t ib = mp2_block(nbf, nocc, occ_block);
  const int64_t nblocks = (nocc + ib - 1) / ib;
  const int64_t ntb_max = ib * nv;
  if (nbf * ntb_max >= (int64_t)1 << 32)
    return fail(c, QSGW_ERR_INVALID_ARG, "mp2: nbf * block transitions must stay below 2^32");
  double *Bia = nullptr, *D = nullptr, *R = nullptr, *E = nullptr;
  CHECK(ws_get(c, W_MP2_BIA, (size_t)(naux * ntr), &Bia));
  CHECK(ws_get(c, W_MP2_D, (size_t)(nn * ntb_max), &D));
  CHECK(ws_get(c, W_MP2_R, (size_t)(nn * ntb_max), &R));
  const int32_t* blocks = nullptr;
  int64_t nblk = 0;
  CHECK(pair_blocks(c, nbf, &blocks, &nblk));
  hipLaunchKernelGGL(k_gather_bia, dim3(blocks_for(naux * ntr)), dim3(256), 0, c->stream, B_mo,
                     (const double*)nullptr, naux, nbf, nocc, Bia, (float*)nullptr);
  CHECK(launch_check(c, "k_gather_bia"));
  if (nblocks > 1) {
    // E[i][n][t] = (in|t) = sum_P B_mo[P][i][n] Bia[P][t]: rows (i, n) are
    // the first nocc nbf entries of each B_mo[P]
    CHECK(ws_get(c, W_MP2_E, (size_t)(nocc * nbf * ntr), &E));
    Strided<false> A{B_mo, 1, nn, 0, nocc * nbf};
    Strided<false> B{Bia, 1, ntr, 0, ntr};
    EpiStore Ep{E, ntr, 0, 0, 1.0};
    Ep.nt = true;
    CHECK((gemm<128, 128, false>(c, "mp2/occ_exchange", A, B, Ep, nocc * nbf, ntr, naux, 1)));
  }
  for (int64_t b = 0; b < nblocks; ++b) {
    const int64_t i0 = b * ib, ni = (nocc - i0 < ib) ? nocc - i0 : ib, ntb = ni * nv;
    {  // D[m][p][tb] = (mp|ia) on pair blocks m <= p, mirrored
      PairRows<8, 16> A{B_mo, nn, 0, nbf, blocks};
      Strided<false> B{Bia + i0 * nv, 1, ntr, 0, ntb};
      EpiPairResidue Ep{D, nullptr, blocks, eps, nullptr, nbf, nocc, ntb, eta};
      CHECK((gemm<128, 128, false>(c, "mp2/direct", A, B, Ep, nblk * 128, ntb, naux, 1)));
    }
    {
      const double* xo = nblocks > 1 ? E : D;
      const int64_t xsn = nblocks > 1 ? ntr : nbf * ntb;
      const int64_t xsi = nblocks > 1 ? nbf * ntr : ntb;
      hipLaunchKernelGGL(k_mp2_rhs_occ, dim3(blocks_for(nbf * nocc * ntb)), dim3(256), 0,
                         c->stream, D, xo, xsn, xsi, eps, nbf, nocc, i0, ni, eta, R);
      CHECK(launch_check(c, "k_mp2_rhs_occ"));
      const int64_t nvt = (nv + 31) / 32;
      hipLaunchKernelGGL(k_mp2_rhs_vir, dim3((unsigned)(nvt * nvt), (unsigned)ni, (unsigned)nbf),
                         dim3(256), 0, c->stream, D, eps, nbf, nocc, i0, ni, eta, R);
      CHECK(launch_check(c, "k_mp2_rhs_vir"));
    }
    {  // G = D Rh^T over k = (p, tb), split over k; V (+)= 1/2 (G + G^T)
      const SplitPlan sp = mp2_split(c->tiles, nbf, ntb);
      double* part = nullptr;
      CHECK(ws_get(c, W_PART, (size_t)(sp.nz * nn), &part));
      Strided<true> A{D, nbf * ntb, 1, 0, nbf};
      Strided<true> B{R, nbf * ntb, 1, 0, nbf};
      EpiStore Ep{part, nbf, 0, nn, 1.0};
      CHECK((gemm_shape<double, false>(c, c->tiles.shape[TU_SIGMA], "mp2/sigma", A, B, Ep, nbf,
                                       nbf, nbf * ntb, 1, sp)));
      CHECK(reduce_sym(c, part, sp.nz, nbf, V, (b > 0 || accumulate) ? 1 : 0));
    }
  }
  return QSGW_OK;
}

}  // namespace

int qsgw_mp2_stage(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                   const double* eps, double eta, double* V, int64_t occ_block, int accumulate) {
  return stage_mp2(c, nbf, naux, nocc, B_mo, eps, eta, V, occ_block, accumulate);
}

extern "C" {

int qsgw_mp2_sigma(qsgw_ctx* c, int64_t nbf, int64_t naux, int64_t nocc, const double* B_mo,
                   const double* eps, double eta, double* V, int64_t occ_block, int accumulate,
                   int precision) {
  CHECK(check_common(c, nbf, naux));
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  if (!(eta > 0.0) || !isfinite(eta)) return fail(c, QSGW_ERR_INVALID_ARG, "need finite eta > 0");
  if (!B_mo || !eps || !V) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  if (occ_block < 0) return fail(c, QSGW_ERR_INVALID_ARG, "need occ_block >= 0");
  if (precision != QSGW_PREC_FP64)
    return fail(c, QSGW_ERR_UNSUPPORTED, "qsgw_mp2_sigma: FP64 only (precision %d)", precision);
  if (nocc * (nbf - nocc) > 0x7fffffffLL)
    return fail(c, QSGW_ERR_INVALID_ARG, "mp2: too many transitions");
  CHECK(check_finite(c, "qsgw_mp2_sigma", {fin(B_mo, naux * nbf * nbf, "B_mo"), fin(eps, nbf, "eps")}));
  CHECK(single_begin(c, kStageSigma));
  CHECK(stage_mp2(c, nbf, naux, nocc, B_mo, eps, eta, V, occ_block, accumulate ? 1 : 0));
  return single_end(c);
}

}  // extern "C"
