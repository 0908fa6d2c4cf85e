// Four-index AO->MO transform, Eq. (16), on explicit integrals (no RI
// factorisation): four quarter transforms, each one FP64 matrix-core GEMM
// over one index, for a slab of the first MO index m:
//   T1[m][nu][lambda][tau] = sum_mu  C[mu][m]      (mu nu|lambda tau)   (M = slab, N = N^3)
//   T2[m][n][lambda][tau]  = sum_nu  C[nu][n]      T1[m][nu][lambda tau] (batched over m)
//   T3[m][n][k][tau]       = sum_lam C[lambda][k]  T2[m][n][lambda][tau] (batched over (m, n))
//   (mn|kl)                = sum_tau T3[m][n][k][tau] C[tau][l]         (M = slab N^2, N = N)
// T1 and T3 live in the context workspace, T2 in the caller's output.
#include "internal.hpp"

extern "C" {

int qsgw_ao2mo_4center(qsgw_ctx* c, int64_t nbf, const double* eri_ao, const double* C,
                       int64_t m_begin, int64_t m_count, double* eri_mo, int precision) {
  CHECK(check_common(c, nbf, 1));
  if (!eri_ao || !C || !eri_mo) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  if (m_begin < 0 || m_count < 1 || m_begin + m_count > nbf)
    return fail(c, QSGW_ERR_INVALID_ARG, "need 0 <= m_begin, m_count >= 1, m_begin + m_count <= nbf");
  if (precision != QSGW_PREC_FP64)
    return fail(c, QSGW_ERR_UNSUPPORTED, "qsgw_ao2mo_4center: FP64 only (precision %d)", precision);
  const int64_t n = nbf, n2 = n * n, n3 = n2 * n;
  if (n > 2000) return fail(c, QSGW_ERR_INVALID_ARG, "nbf too large for the four-index tensor");
  CHECK(check_finite(c, "qsgw_ao2mo_4center", {fin(eri_ao, n3 * n, "eri_ao"), fin(C, n2, "C")}));
  double* T = nullptr;
  CHECK(ws_get(c, W_AO2MO, (size_t)(m_count * n3), &T));
  CHECK(single_begin(c, kStageMo));
  {  // quarter 1: T[m][x] = sum_mu C[mu][m_begin + m] eri[mu][x]
    Strided<false> A{C + m_begin, 1, n, 0, m_count};
    Strided<false> B{eri_ao, 1, n3, 0, n3};
    EpiStore E{T, n3, 0, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "ao2mo/q1", A, B, E, m_count, n3, n, 1)));
  }
  {  // quarter 2, per m: out[m][q][y] = sum_nu C[nu][q] T[m][nu][y]
    Strided<false> A{C, 1, n, 0, n};
    Strided<false> B{T, 1, n2, n3, n2};
    EpiStore E{eri_mo, n2, n3, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "ao2mo/q2", A, B, E, n, n2, n, m_count)));
  }
  {  // quarter 3, per (m, q): T[mq][k][tau] = sum_lambda C[lambda][k] out[mq][lambda][tau]
    Strided<false> A{C, 1, n, 0, n};
    Strided<false> B{eri_mo, 1, n, n2, n};
    EpiStore E{T, n, n2, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "ao2mo/q3", A, B, E, n, n, n, m_count * n)));
  }
  {  // quarter 4: out[mqk][l] = sum_tau T[mqk][tau] C[tau][l]
    Strided<true> A{T, n, 1, 0, m_count * n2};
    Strided<false> B{C, 1, n, 0, n};
    EpiStore E{eri_mo, n, 0, 0, 1.0};
    CHECK((gemm<64, 64, false>(c, "ao2mo/q4", A, B, E, m_count * n2, n, n, 1)));
  }
  return single_end(c);
}

}  // extern "C"
