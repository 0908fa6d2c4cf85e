// Allocation-free variant of the qsGW matrix product (qsgw_sigma with
// QSGW_SIGMA_QS_MATRIX, Eqs. (17) and (19)) for callers that cannot allocate
// device memory.  Its K-split partial sums and its finite-input flag live in
// one file-scope device array of fixed size instead of the context's
// workspace; every other step is the same product and the same deterministic
// symmetrising reduction as the allocating entry point.
#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB on every device the library runs on
constexpr int64_t kScratchDoubles = (int64_t)(kScratchBytes / sizeof(double));
constexpr int64_t kFlagDoubles = 32;  // the first 256 bytes: the finite-input flag word
constexpr int64_t kMaxSlices = 64;    // one-level symmetrising reduction (no second buffer)

// Host code never passes this name to a kernel: it is a host-side stand-in.
// Kernels receive the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

}  // namespace

// Looks up the current device's copy of `scratch` (once per device, with that
// device current) and stores it in the context.
int noalloc_setup(qsgw_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return fail(c, QSGW_ERR_UNSUPPORTED, "device index %d out of range", c->device);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[c->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, QSGW_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[c->device] = static_cast<double*>(p);
  }
  c->scratch = g_scratch[c->device];
  return QSGW_OK;
}

extern "C" {

int qsgw_sigma_qs_noalloc(qsgw_ctx* c, int64_t nbf, int64_t nocc, int64_t ns, const double* w,
                          const double* wh, const double* eps, const double* Omega, double eta,
                          double* out, int accumulate) {
  CHECK(check_common(c, nbf, 1));
  if (!(nocc > 0 && nocc < nbf)) return fail(c, QSGW_ERR_INVALID_ARG, "need 0 < nocc < nbf");
  if (ns < 1) return fail(c, QSGW_ERR_INVALID_ARG, "need ns >= 1");
  if (!(eta > 0.0) || !isfinite(eta)) return fail(c, QSGW_ERR_INVALID_ARG, "need finite eta > 0");
  if (!w || !eps || !Omega || !out) return fail(c, QSGW_ERR_INVALID_ARG, "null pointer");
  if (!c->scratch) return fail(c, QSGW_ERR_HIP, "the device scratch array was not set up");
  const int64_t nn = nbf * nbf;
  const int64_t fit = (kScratchDoubles - kFlagDoubles) / nn;
  if (fit < 1)
    return fail(c, QSGW_ERR_INVALID_ARG,
                "qsgw_sigma_qs_noalloc: one %lld x %lld partial sum exceeds the %zu-byte scratch "
                "(nbf <= %lld)",
                (long long)nbf, (long long)nbf, kScratchBytes,
                (long long)sqrt((double)(kScratchDoubles - kFlagDoubles)));
  if (nbf * ns >= (int64_t)1 << 32)
    return fail(c, QSGW_ERR_INVALID_ARG, "sigma: nbf * ns must stay below 2^32");

  // finite inputs: one flag word at the front of the scratch, cleared by a kernel
  int* flag = reinterpret_cast<int*>(c->scratch);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, c->stream, flag);
  const FiniteArg args[4] = {fin(w, nn * ns, "w"), fin(wh, nn * ns, "wh"), fin(eps, nbf, "eps"),
                             fin(Omega, ns, "Omega")};
  for (int a = 0; a < 4; ++a) {
    if (!args[a].p) continue;
    const int64_t nb = (args[a].n + 255) / 256;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0,
                       c->stream, static_cast<const double*>(args[a].p), args[a].n, flag, 1 << a);
  }
  CHECK(launch_check(c, "k_check_finite"));
  int mask = 0;
  HIP_TRY(c, hipMemcpyAsync(&mask, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int a = 0; a < 4; ++a)
    if (mask & (1 << a))
      return fail(c, QSGW_ERR_NONFINITE, "qsgw_sigma_qs_noalloc: non-finite value in %s",
                  args[a].name);

  // the K-split of qsgw_sigma, capped by what the scratch holds
  SplitPlan sp = sigma_split(c->tiles, nbf, ns);
  const int64_t zmax = fit < kMaxSlices ? fit : kMaxSlices;
  if (sp.nz > zmax) sp = split_plan(nbf * ns, zmax);
  double* part = c->scratch + kFlagDoubles;
  Strided<true> B{w, nbf * ns, 1, 0, nbf};
  EpiStore E{part, nbf, 0, nn, 1.0};
  if (wh) {
    Strided<true> A{wh, nbf * ns, 1, 0, nbf};
    CHECK((gemm_shape<double, false>(c, c->tiles.shape[TU_SIGMA], "sigma_qs_noalloc", A, B, E, nbf,
                                     nbf, nbf * ns, 1, sp)));
  } else {
    PoleScaledResidueOp A{w, eps, Omega, nbf, nocc, ns, eta};
    CHECK((gemm_shape<double, false>(c, c->tiles.shape[TU_SIGMA], "sigma_qs_noalloc", A, B, E, nbf,
                                     nbf, nbf * ns, 1, sp)));
  }
  hipLaunchKernelGGL(k_reduce_sym, dim3(blocks_for(nn)), dim3(256), 0, c->stream, part, sp.nz, nbf,
                     out, accumulate ? 1 : 0);
  return launch_check(c, "k_reduce_sym");
}

}  // extern "C"
