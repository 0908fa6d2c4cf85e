"""ctypes binding of libqsgw (include/qsgw.h).

Argument marshalling only: every function checks that its torch tensors are
HIP-device, float64 (int64 for state lists), contiguous and of the expected
shape, then passes raw device pointers and the context's stream to the C-ABI
entry point of the same name.  No arithmetic of the method happens here.  If
the compiled library is missing the import of this module fails.
"""
from __future__ import annotations

import ctypes as ct
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsgw.so")

OK = 0
NOT_CONVERGED = 1
ERR_INVALID_ARG = -1
ERR_NONFINITE = -2
ERR_HIP = -3
ERR_SOLVER = -4
ERR_ALLOC = -5
ERR_UNSUPPORTED = -6

PREC_FP64 = 0
PREC_FP32 = 1
PREC_SPLIT_BF16 = 2

SIGMA_QS_MATRIX = 0
SIGMA_DIAG_GRID = 1
SIGMA_DIAG_SELF = 2

FOCK_FULL_JK = 0
FOCK_FROZEN = 1
OPT_GRAPH = 1
OPT_REFINE = 2
OPT_QSMP2 = 4
OPT_REPLAY_EIG = 8
EIG_AUTO = 0
EIG_ROCSOLVER = 1
EIG_TWO_STAGE = 2
REPORT_MAX_ITERS = 64
MLP_NPARAMS = 18817
MLP_NFEAT = 16
STAGES = ("mo_transform", "rpa_build", "eig_rpa", "residues", "sigma", "fock", "eig_fock")

EXPORTS = ("qsgw_version", "qsgw_ctx_create", "qsgw_ctx_destroy", "qsgw_last_error",
           "qsgw_last_stage_ms", "qsgw_mo_transform", "qsgw_rpa_build", "qsgw_rpa_solve",
           "qsgw_residues", "qsgw_sigma", "qsgw_mp2_sigma", "qsgw_ao2mo_4center",
           "qsgw_gw_unrestricted", "qsgw_fock_unrestricted", "qsgw_hf_core", "qsgw_iterate",
           "qsgw_iterate_batched", "qsgw_mlp_features", "qsgw_mlp_forward",
           "qsgw_mlp_train_step", "qsgw_warm_start", "qsgw_set_tiles", "qsgw_get_tiles",
           "qsgw_set_eigensolver", "qsgw_sigma_qs_noalloc", "qsgw_iterate_unrestricted",
           "qsgw_mlp_forward_bf16")


class QsgwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libqsgw error {code}: {msg}")
        self.code = code


class Problem(ct.Structure):
    _fields_ = [("nbf", ct.c_int64), ("naux", ct.c_int64), ("nocc", ct.c_int64),
                ("B_ao", ct.c_void_p), ("h", ct.c_void_p)]


class State(ct.Structure):
    _fields_ = [("eps", ct.c_void_p), ("C", ct.c_void_p), ("Vc", ct.c_void_p),
                ("iteration", ct.c_int64), ("diag", ct.c_void_p)]


class Options(ct.Structure):
    _fields_ = [("precision", ct.c_int), ("eta", ct.c_double), ("tol", ct.c_double),
                ("max_iter", ct.c_int64), ("mix", ct.c_double), ("fock_mode", ct.c_int),
                ("s_block", ct.c_int64), ("flags", ct.c_int64), ("near_pole", ct.c_double),
                ("warm_start", ct.c_void_p), ("diis", ct.c_int64)]


KERNELS = ("mo_transform_1", "mo_transform_2", "casida", "residue_rho", "residue_w",
           "sigma_qs_gemm", "sigma_qs_reduce", "fock")


class Report(ct.Structure):
    _fields_ = [("iterations", ct.c_int64), ("converged", ct.c_int),
                ("max_deps", ct.c_double * REPORT_MAX_ITERS), ("ms_stage", ct.c_double * 7),
                ("hot_flops", ct.c_double), ("ms_kernel", ct.c_double * 8),
                ("kernel_flops", ct.c_double * 8), ("kernel_launches", ct.c_int64 * 8)]

    def as_dict(self):
        n = min(self.iterations, REPORT_MAX_ITERS)
        return dict(iterations=int(self.iterations), converged=bool(self.converged),
                    max_deps=[self.max_deps[i] for i in range(n)],
                    ms=dict(zip(STAGES, list(self.ms_stage))), hot_flops=self.hot_flops,
                    kernel_ms=dict(zip(KERNELS, list(self.ms_kernel))),
                    kernel_flops=dict(zip(KERNELS, list(self.kernel_flops))),
                    kernel_launches=dict(zip(KERNELS, [int(x) for x in self.kernel_launches])))


def load_library(path: str = LIB_PATH) -> ct.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2210_17093_amd.build`")
    lib = ct.CDLL(path)
    P, I64, D, I = ct.c_void_p, ct.c_int64, ct.c_double, ct.c_int
    sig = {
        "qsgw_version": ([], I),
        "qsgw_ctx_create": ([ct.POINTER(P), P], I),
        "qsgw_ctx_destroy": ([P], I),
        "qsgw_last_error": ([P], ct.c_char_p),
        "qsgw_last_stage_ms": ([P, ct.POINTER(D), I], I),
        "qsgw_mo_transform": ([P, I64, I64, P, P, P, I], I),
        "qsgw_rpa_build": ([P, I64, I64, I64, P, P, P, P, I], I),
        "qsgw_rpa_solve": ([P, I64, P, P], I),
        "qsgw_residues": ([P, I64, I64, I64, P, P, P, P, I64, I64, P, P, P, D, I], I),
        "qsgw_sigma": ([P, I, I64, I64, I64, P, P, P, P, D, P, I64, P, I64, P, I], I),
        "qsgw_hf_core": ([P, I64, I64, I64, P, P, P, P], I),
        "qsgw_mp2_sigma": ([P, I64, I64, I64, P, P, D, P, I64, I, I], I),
        "qsgw_ao2mo_4center": ([P, I64, P, P, I64, I64, P, I], I),
        "qsgw_gw_unrestricted": ([P, I64, I64, I64, I64, P, P, P, P, D, P, P, P, I], I),
        "qsgw_fock_unrestricted": ([P, I64, I64, I64, I64, P, P, P, P, P, P, P, P, P], I),
        "qsgw_iterate": ([P, ct.POINTER(Problem), ct.POINTER(State), ct.POINTER(Options),
                          ct.POINTER(Report)], I),
        "qsgw_iterate_unrestricted": ([P, ct.POINTER(Problem), I64, ct.POINTER(State),
                                       ct.POINTER(State), ct.POINTER(Options), ct.POINTER(Report)], I),
        "qsgw_iterate_batched": ([P, I64, ct.POINTER(Problem), ct.POINTER(State),
                                  ct.POINTER(Options), ct.POINTER(Report)], I),
        "qsgw_mlp_features": ([P, I64, I64, P, P, P, P, P], I),
        "qsgw_mlp_forward": ([P, P, I64, P, P], I),
        "qsgw_mlp_forward_bf16": ([P, P, I64, P, P], I),
        "qsgw_mlp_train_step": ([P, P, P, P, I64, D, I64, P, P, P, P], I),
        "qsgw_warm_start": ([P, I64, P, P, P, P, P], I),
        "qsgw_set_tiles": ([P, ct.c_char_p], I),
        "qsgw_get_tiles": ([P, ct.c_char_p, I64], I),
        "qsgw_set_eigensolver": ([P, I], I),
        "qsgw_sigma_qs_noalloc": ([P, I64, I64, I64, P, P, P, P, D, P, I], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = load_library()


def lib() -> ct.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _ptr(t: torch.Tensor, shape, dtype=torch.float64, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ct.c_void_p(t.data_ptr())


class Context:
    """A libqsgw context bound to a torch HIP stream (the current one by default)."""

    def __init__(self, stream: torch.cuda.Stream | None = None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ct.c_void_p()
        rc = lib().qsgw_ctx_create(ct.byref(h), ct.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise QsgwError(rc, "qsgw_ctx_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().qsgw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_tiles(self, spec: str | None):
        """Tile table of the context (see qsgw_set_tiles); None restores defaults."""
        self.check(lib().qsgw_set_tiles(self.handle, spec.encode() if spec else None))

    def set_eigensolver(self, solver: int):
        """Casida eigensolver of the context (EIG_AUTO, EIG_ROCSOLVER, EIG_TWO_STAGE)."""
        self.check(lib().qsgw_set_eigensolver(self.handle, int(solver)))

    def get_tiles(self) -> str:
        buf = ct.create_string_buffer(512)
        self.check(lib().qsgw_get_tiles(self.handle, buf, 512))
        return buf.value.decode()

    def check(self, rc, allow=(OK,)):
        if rc in allow:
            return rc
        msg = lib().qsgw_last_error(self.handle)
        raise QsgwError(rc, msg.decode() if msg else "")

    def last_stage_ms(self):
        buf = (ct.c_double * 7)()
        self.check(lib().qsgw_last_stage_ms(self.handle, buf, 7))
        return dict(zip(STAGES, list(buf)))


def qsgw_version() -> int:
    return lib().qsgw_version()


def qsgw_mo_transform(ctx: Context, B_ao, C, B_mo=None, precision=PREC_FP64):
    naux, nbf, _ = B_ao.shape
    if B_mo is None:
        B_mo = torch.empty_like(B_ao)
    ctx.check(lib().qsgw_mo_transform(ctx.handle, nbf, naux, _ptr(B_ao, (naux, nbf, nbf), name="B_ao"),
                                      _ptr(C, (nbf, nbf), name="C"),
                                      _ptr(B_mo, (naux, nbf, nbf), name="B_mo"), precision))
    return B_mo


def qsgw_rpa_build(ctx: Context, B_mo, eps, nocc, M=None, sqrt_delta=None, precision=PREC_FP64):
    naux, nbf, _ = B_mo.shape
    ntr = nocc * (nbf - nocc)
    if M is None:
        M = torch.empty((ntr, ntr), dtype=torch.float64, device=B_mo.device)
    if sqrt_delta is None:
        sqrt_delta = torch.empty(ntr, dtype=torch.float64, device=B_mo.device)
    ctx.check(lib().qsgw_rpa_build(ctx.handle, nbf, naux, nocc,
                                   _ptr(B_mo, (naux, nbf, nbf), name="B_mo"),
                                   _ptr(eps, (nbf,), name="eps"), _ptr(M, (ntr, ntr), name="M"),
                                   _ptr(sqrt_delta, (ntr,), name="sqrt_delta"), precision))
    return M, sqrt_delta


def qsgw_rpa_solve(ctx: Context, M_to_Z, Omega=None):
    ntr = M_to_Z.shape[0]
    if Omega is None:
        Omega = torch.empty(ntr, dtype=torch.float64, device=M_to_Z.device)
    ctx.check(lib().qsgw_rpa_solve(ctx.handle, ntr, _ptr(M_to_Z, (ntr, ntr), name="M"),
                                   _ptr(Omega, (ntr,), name="Omega")))
    return M_to_Z, Omega


def qsgw_residues(ctx: Context, B_mo, sqrt_delta, Z, Omega, nocc, s_begin=0, s_count=None,
                  w=None, precision=PREC_FP64, weighted=False, eps=None, eta=0.0):
    """Residues w of excitations [s_begin, s_begin + s_count).  With weighted=True
    also returns the pole-weighted copy wh (needs eps and eta): (w, wh)."""
    naux, nbf, _ = B_mo.shape
    ntr = nocc * (nbf - nocc)
    if s_count is None:
        s_count = ntr - s_begin
    if w is None:
        w = torch.empty((nbf, nbf, s_count), dtype=torch.float64, device=B_mo.device)
    wh = None
    if weighted:
        wh = torch.empty((nbf, nbf, s_count), dtype=torch.float64, device=B_mo.device)
    ctx.check(lib().qsgw_residues(ctx.handle, nbf, naux, nocc,
                                  _ptr(B_mo, (naux, nbf, nbf), name="B_mo"),
                                  _ptr(sqrt_delta, (ntr,), name="sqrt_delta"),
                                  _ptr(Z, (ntr, ntr), name="Z"), _ptr(Omega, (ntr,), name="Omega"),
                                  s_begin, s_count, _ptr(w, (nbf, nbf, s_count), name="w"),
                                  _ptr(wh, (nbf, nbf, s_count), name="wh") if weighted else None,
                                  _ptr(eps, (nbf,), name="eps") if weighted else None,
                                  float(eta), precision))
    return (w, wh) if weighted else w


def qsgw_sigma_qs(ctx: Context, w, eps, Omega_block, nocc, eta, out=None, accumulate=False,
                  wh=None):
    nbf, _, ns = w.shape
    if out is None:
        out = torch.empty((nbf, nbf), dtype=torch.float64, device=w.device)
    ctx.check(lib().qsgw_sigma(ctx.handle, SIGMA_QS_MATRIX, nbf, nocc, ns,
                               _ptr(w, (nbf, nbf, ns), name="w"),
                               _ptr(wh, (nbf, nbf, ns), name="wh") if wh is not None else None,
                               _ptr(eps, (nbf,), name="eps"),
                               _ptr(Omega_block, (ns,), name="Omega"), float(eta), None, 0, None, 0,
                               _ptr(out, (nbf, nbf), name="out"), int(bool(accumulate))))
    return out


def qsgw_sigma_qs_noalloc(ctx: Context, w, eps, Omega_block, nocc, eta, out, accumulate=False,
                          wh=None):
    """qsGW matrix (QSGW_SIGMA_QS_MATRIX) through the allocation-free entry
    point: `out` must be given (the call allocates nothing)."""
    nbf, _, ns = w.shape
    ctx.check(lib().qsgw_sigma_qs_noalloc(ctx.handle, nbf, nocc, ns,
                                          _ptr(w, (nbf, nbf, ns), name="w"),
                                          _ptr(wh, (nbf, nbf, ns), name="wh") if wh is not None else None,
                                          _ptr(eps, (nbf,), name="eps"),
                                          _ptr(Omega_block, (ns,), name="Omega"), float(eta),
                                          _ptr(out, (nbf, nbf), name="out"), int(bool(accumulate))))
    return out


def qsgw_sigma_diag(ctx: Context, w, eps, Omega_block, nocc, eta, omega, states, out=None,
                    accumulate=False):
    """Returns complex128 [nstates][nomega] (a view of the interleaved float64 buffer)."""
    nbf, _, ns = w.shape
    nomega, nstates = omega.shape[0], states.shape[0]
    if out is None:
        out = torch.empty((nstates, nomega, 2), dtype=torch.float64, device=w.device)
    ctx.check(lib().qsgw_sigma(ctx.handle, SIGMA_DIAG_GRID, nbf, nocc, ns,
                               _ptr(w, (nbf, nbf, ns), name="w"), None,
                               _ptr(eps, (nbf,), name="eps"),
                               _ptr(Omega_block, (ns,), name="Omega"), float(eta),
                               _ptr(omega, (nomega,), name="omega"), nomega,
                               _ptr(states, (nstates,), torch.int64, name="states"), nstates,
                               _ptr(out, (nstates, nomega, 2), name="out"), int(bool(accumulate))))
    return torch.view_as_complex(out)


def qsgw_sigma_diag_self(ctx: Context, w, eps, Omega_block, nocc, eta, states, out=None,
                         accumulate=False):
    """Per-state Eq. (17) at omega = eps_m: float64 [nstates][3] holding
    Re Sigma_mm(eps_m), Im Sigma_mm(eps_m), Re dSigma_mm/domega(eps_m)."""
    nbf, _, ns = w.shape
    nstates = states.shape[0]
    if out is None:
        out = torch.empty((nstates, 3), dtype=torch.float64, device=w.device)
    ctx.check(lib().qsgw_sigma(ctx.handle, SIGMA_DIAG_SELF, nbf, nocc, ns,
                               _ptr(w, (nbf, nbf, ns), name="w"), None,
                               _ptr(eps, (nbf,), name="eps"),
                               _ptr(Omega_block, (ns,), name="Omega"), float(eta), None, 0,
                               _ptr(states, (nstates,), torch.int64, name="states"), nstates,
                               _ptr(out, (nstates, 3), name="out"), int(bool(accumulate))))
    return out


def qsgw_mp2_sigma(ctx: Context, B_mo, eps, nocc, eta, out=None, occ_block=0, accumulate=False,
                   precision=PREC_FP64):
    naux, nbf, _ = B_mo.shape
    if out is None:
        out = torch.empty((nbf, nbf), dtype=torch.float64, device=B_mo.device)
    ctx.check(lib().qsgw_mp2_sigma(ctx.handle, nbf, naux, nocc,
                                   _ptr(B_mo, (naux, nbf, nbf), name="B_mo"),
                                   _ptr(eps, (nbf,), name="eps"), float(eta),
                                   _ptr(out, (nbf, nbf), name="out"), int(occ_block),
                                   int(bool(accumulate)), int(precision)))
    return out


def qsgw_ao2mo_4center(ctx: Context, eri_ao, C, m_begin=0, m_count=None, out=None,
                       precision=PREC_FP64):
    nbf = C.shape[0]
    m_count = nbf - m_begin if m_count is None else m_count
    if out is None:
        out = torch.empty((m_count, nbf, nbf, nbf), dtype=torch.float64, device=C.device)
    ctx.check(lib().qsgw_ao2mo_4center(ctx.handle, nbf, _ptr(eri_ao, (nbf,) * 4, name="eri_ao"),
                                       _ptr(C, (nbf, nbf), name="C"), int(m_begin), int(m_count),
                                       _ptr(out, (m_count, nbf, nbf, nbf), name="out"),
                                       int(precision)))
    return out


def qsgw_gw_unrestricted(ctx: Context, B_mo_a, B_mo_b, eps_a, eps_b, nocc_a, nocc_b, eta,
                         precision=PREC_FP64):
    """Open-shell GW potential of each spin; returns (V_a, V_b, Omega)."""
    naux, nbf, _ = B_mo_a.shape
    ntr = nocc_a * (nbf - nocc_a) + nocc_b * (nbf - nocc_b)
    V_a = torch.empty((nbf, nbf), dtype=torch.float64, device=B_mo_a.device)
    V_b = torch.empty_like(V_a)
    Om = torch.empty((ntr,), dtype=torch.float64, device=B_mo_a.device)
    ctx.check(lib().qsgw_gw_unrestricted(ctx.handle, nbf, naux, int(nocc_a), int(nocc_b),
                                         _ptr(B_mo_a, (naux, nbf, nbf), name="B_mo_a"),
                                         _ptr(B_mo_b, (naux, nbf, nbf), name="B_mo_b"),
                                         _ptr(eps_a, (nbf,), name="eps_a"),
                                         _ptr(eps_b, (nbf,), name="eps_b"), float(eta),
                                         _ptr(V_a, (nbf, nbf), name="V_a"),
                                         _ptr(V_b, (nbf, nbf), name="V_b"),
                                         _ptr(Om, (ntr,), name="Omega"), int(precision)))
    return V_a, V_b, Om


def qsgw_fock_unrestricted(ctx: Context, B_mo_a, B_mo_b, h, V_a, V_b, nocc_a, nocc_b, eps_a, eps_b,
                           C_a, C_b):
    """Open-shell Fock update: eps_a, eps_b (out) and C_a, C_b (in/out) in place."""
    naux, nbf, _ = B_mo_a.shape
    sq = (nbf, nbf)
    ctx.check(lib().qsgw_fock_unrestricted(ctx.handle, nbf, naux, int(nocc_a), int(nocc_b),
                                           _ptr(B_mo_a, (naux, nbf, nbf), name="B_mo_a"),
                                           _ptr(B_mo_b, (naux, nbf, nbf), name="B_mo_b"),
                                           _ptr(h, sq, name="h"), _ptr(V_a, sq, name="V_a"),
                                           _ptr(V_b, sq, name="V_b"),
                                           _ptr(eps_a, (nbf,), name="eps_a"),
                                           _ptr(eps_b, (nbf,), name="eps_b"),
                                           _ptr(C_a, sq, name="C_a"), _ptr(C_b, sq, name="C_b")))
    return eps_a, eps_b, C_a, C_b


def qsgw_hf_core(ctx: Context, B_ao, C0, eps0, nocc, h=None):
    naux, nbf, _ = B_ao.shape
    if h is None:
        h = torch.empty((nbf, nbf), dtype=torch.float64, device=B_ao.device)
    ctx.check(lib().qsgw_hf_core(ctx.handle, nbf, naux, nocc, _ptr(B_ao, (naux, nbf, nbf), name="B_ao"),
                                 _ptr(C0, (nbf, nbf), name="C0"), _ptr(eps0, (nbf,), name="eps0"),
                                 _ptr(h, (nbf, nbf), name="h")))
    return h


def qsgw_iterate(ctx: Context, B_ao, h, nocc, eps, C, eta, tol=1e-6, max_iter=1, mix=1.0,
                 Vc=None, iteration=0, s_block=0, precision=PREC_FP64, diag=None, refine=False,
                 near_pole=0.0, qsmp2=False, fock_mode=FOCK_FULL_JK, warm_start=None,
                 replay_eig=False, diis=0):
    """Runs qsGW iterations (qsMP2 iterations with qsmp2=True) in place on (eps, C).
    warm_start: None or a float32 [nbf] device tensor of predicted shifts.
    replay_eig: reuse the context's last Casida eigenpairs (QSGW_OPT_REPLAY_EIG).
    diis: 0, or the DIIS subspace size (2..16) of qsgw_options.diis.
    Returns (status, report dict, iteration)."""
    naux, nbf, _ = B_ao.shape
    prob = Problem(nbf, naux, nocc, _ptr(B_ao, (naux, nbf, nbf), name="B_ao"),
                   _ptr(h, (nbf, nbf), name="h"))
    st = State(_ptr(eps, (nbf,), name="eps"), _ptr(C, (nbf, nbf), name="C"),
               _ptr(Vc, (nbf, nbf), name="Vc") if Vc is not None else None, iteration,
               _ptr(diag, (nbf, 4), name="diag") if diag is not None else None)
    flags = ((OPT_REFINE if refine else 0) | (OPT_QSMP2 if qsmp2 else 0)
             | (OPT_REPLAY_EIG if replay_eig else 0))
    opt = Options(precision, float(eta), float(tol), int(max_iter), float(mix), int(fock_mode),
                  int(s_block), flags, float(near_pole),
                  _ptr(warm_start, (nbf,), torch.float32, "warm_start")
                  if warm_start is not None else None, int(diis))
    rep = Report()
    rc = ctx.check(lib().qsgw_iterate(ctx.handle, ct.byref(prob), ct.byref(st), ct.byref(opt),
                                      ct.byref(rep)), allow=(OK, NOT_CONVERGED))
    return rc, rep.as_dict(), int(st.iteration)


def qsgw_iterate_unrestricted(ctx: Context, B_ao, h, nocc_a, nocc_b, eps_a, C_a, eps_b, C_b, eta,
                              tol=1e-6, max_iter=1, iteration=0):
    """Open-shell qsGW iterations in place on (eps_a, C_a) and (eps_b, C_b).
    Returns (status, report dict, iteration)."""
    naux, nbf, _ = B_ao.shape
    prob = Problem(nbf, naux, nocc_a, _ptr(B_ao, (naux, nbf, nbf), name="B_ao"),
                   _ptr(h, (nbf, nbf), name="h"))
    sa = State(_ptr(eps_a, (nbf,), name="eps_a"), _ptr(C_a, (nbf, nbf), name="C_a"), None,
               iteration, None)
    sb = State(_ptr(eps_b, (nbf,), name="eps_b"), _ptr(C_b, (nbf, nbf), name="C_b"), None,
               iteration, None)
    opt = Options(PREC_FP64, float(eta), float(tol), int(max_iter), 1.0, FOCK_FULL_JK, 0, 0, 0.0,
                  None)
    rep = Report()
    rc = ctx.check(lib().qsgw_iterate_unrestricted(ctx.handle, ct.byref(prob), int(nocc_b),
                                                   ct.byref(sa), ct.byref(sb), ct.byref(opt),
                                                   ct.byref(rep)), allow=(OK, NOT_CONVERGED))
    return rc, rep.as_dict(), int(sa.iteration)


def qsgw_iterate_batched(ctx: Context, mols, eta, tol=1e-6, max_iter=1, graph=False,
                         precision=PREC_FP64, mix=1.0):
    """Batched qsGW iterations in place.  `mols` is a sequence of dicts with
    device tensors B_ao [naux][nbf][nbf], h, eps, C, the int nocc, and
    optionally Vc [nbf][nbf] (required when mix != 1), diag [nbf][4] and
    iteration.  Returns (status, list of report dicts)."""
    n = len(mols)
    if n < 1:
        raise ValueError("need at least one molecule")
    probs = (Problem * n)()
    states = (State * n)()
    for i, m in enumerate(mols):
        naux, nbf, _ = m["B_ao"].shape
        probs[i] = Problem(nbf, naux, int(m["nocc"]), _ptr(m["B_ao"], (naux, nbf, nbf), name="B_ao"),
                           _ptr(m["h"], (nbf, nbf), name="h"))
        Vc, diag = m.get("Vc"), m.get("diag")
        states[i] = State(_ptr(m["eps"], (nbf,), name="eps"), _ptr(m["C"], (nbf, nbf), name="C"),
                          _ptr(Vc, (nbf, nbf), name="Vc") if Vc is not None else None,
                          int(m.get("iteration", 0)),
                          _ptr(diag, (nbf, 4), name="diag") if diag is not None else None)
    opt = Options(precision, float(eta), float(tol), int(max_iter), float(mix), FOCK_FULL_JK, 0,
                  OPT_GRAPH if graph else 0)
    reps = (Report * n)()
    rc = ctx.check(lib().qsgw_iterate_batched(ctx.handle, n, probs, states, ct.byref(opt), reps),
                   allow=(OK, NOT_CONVERGED))
    for i, m in enumerate(mols):
        m["iteration"] = int(states[i].iteration)
    return rc, [r.as_dict() for r in reps]


# ------------------------------------------------------------ warm start --
def qsgw_mlp_features(ctx: Context, eps, diag, nocc, mean=None, scale=None, out=None):
    """Per-state features [nbf][16] (float32) of one molecule."""
    nbf = eps.shape[0]
    if out is None:
        out = torch.empty((nbf, MLP_NFEAT), dtype=torch.float32, device=eps.device)
    ctx.check(lib().qsgw_mlp_features(
        ctx.handle, nbf, int(nocc), _ptr(eps, (nbf,), name="eps"), _ptr(diag, (nbf, 4), name="diag"),
        _ptr(mean, (MLP_NFEAT,), torch.float32, name="mean") if mean is not None else None,
        _ptr(scale, (MLP_NFEAT,), torch.float32, name="scale") if scale is not None else None,
        _ptr(out, (nbf, MLP_NFEAT), torch.float32, name="X")))
    return out


def qsgw_mlp_forward(ctx: Context, params, X, out=None, bf16=False):
    """Network outputs for the rows of X; bf16=True runs the BF16 inference
    entry point (qsgw_mlp_forward_bf16)."""
    n = X.shape[0]
    if out is None:
        out = torch.empty((n,), dtype=torch.float32, device=X.device)
    fn = lib().qsgw_mlp_forward_bf16 if bf16 else lib().qsgw_mlp_forward
    ctx.check(fn(ctx.handle, _ptr(params, (MLP_NPARAMS,), torch.float32, "params"),
                 n, _ptr(X, (n, MLP_NFEAT), torch.float32, "X"), _ptr(out, (n,), torch.float32, "y")))
    return out


def qsgw_mlp_forward_bf16(ctx: Context, params, X, out=None):
    """BF16 inference of the network (qsgw_mlp_forward_bf16)."""
    return qsgw_mlp_forward(ctx, params, X, out, bf16=True)


def qsgw_mlp_train_step(ctx: Context, params, adam_m, adam_v, step, lr, X, target, grad=None,
                        loss=None):
    """One Adam step in place; returns (grad, loss) device tensors when given."""
    n = X.shape[0]
    f32 = torch.float32
    ctx.check(lib().qsgw_mlp_train_step(
        ctx.handle, _ptr(params, (MLP_NPARAMS,), f32, "params"), _ptr(adam_m, (MLP_NPARAMS,), f32, "m"),
        _ptr(adam_v, (MLP_NPARAMS,), f32, "v"), int(step), float(lr), n,
        _ptr(X, (n, MLP_NFEAT), f32, "X"), _ptr(target, (n,), f32, "target"),
        _ptr(grad, (MLP_NPARAMS,), f32, "grad") if grad is not None else None,
        _ptr(loss, (1,), torch.float64, "loss") if loss is not None else None))
    return grad, loss


def qsgw_warm_start(ctx: Context, eps0, C0, delta, eps=None, C=None):
    nbf = eps0.shape[0]
    if eps is None:
        eps = torch.empty_like(eps0)
    if C is None:
        C = torch.empty_like(C0)
    ctx.check(lib().qsgw_warm_start(ctx.handle, nbf, _ptr(eps0, (nbf,), name="eps0"),
                                    _ptr(C0, (nbf, nbf), name="C0"),
                                    _ptr(delta, (nbf,), torch.float32, "delta"),
                                    _ptr(eps, (nbf,), name="eps"), _ptr(C, (nbf, nbf), name="C")))
    return eps, C
