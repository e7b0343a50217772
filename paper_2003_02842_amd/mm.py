"""Python binding of libmm.so: argument marshalling only.

Every step of the computation runs in the library's gfx950 kernels; this module
checks tensor types, allocates outputs and workspace with PyTorch (device memory
only) and passes raw pointers and the current HIP stream through the C ABI
declared in ``include/mm.h``.  There is no fallback: without the built library
every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmm.so")

MM_OK, MM_ERR_ARG, MM_ERR_DATA, MM_ERR_TOL, MM_ERR_WORKSPACE, MM_ERR_HIP, MM_ERR_UNSUPPORTED = range(7)
DIRICHLET, FEJER = 0, 1
GAUSSIAN, KAISER_BESSEL, ES = 0, 1, 2
PLAIN_FP64, MIXED = 0, 1

_KERNELS = {"gaussian": GAUSSIAN, "g": GAUSSIAN, "fgg": GAUSSIAN, "kaiser_bessel": KAISER_BESSEL,
            "kb": KAISER_BESSEL, "es": ES}
_BASES = {"dirichlet": DIRICHLET, "fejer": FEJER}
_PRECS = {"fp64": PLAIN_FP64, "plain": PLAIN_FP64, "mixed": MIXED}

EXPORTED = ["mm_plan_query", "mm_nufft1_workspace_size", "mm_nufft1", "mm_cov_workspace_size", "mm_cov",
            "mm_estimate_workspace_size", "mm_estimate", "mm_estimate_noalloc", "mm_graph_cache_clear",
            "mm_matrix_to_csr_workspace_size", "mm_matrix_to_csr", "mm_snap_times",
            "mm_cov_pairwise_workspace_size", "mm_cov_pairwise",
            "mm_status_string", "mm_profile_enable", "mm_profile_read", "mm_profile_reset"]


class MMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (where, _status_text(status), status))


class CsrInfo(ctypes.Structure):
    _fields_ = [("E", ctypes.c_int64), ("N", ctypes.c_int32), ("t0", ctypes.c_double), ("T", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("sigma", ctypes.c_double), ("tile", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("es_beta_per_tap", ctypes.c_double), ("fft_generic", ctypes.c_int32),
                ("spread_direct", ctypes.c_int32), ("syrk_tile", ctypes.c_int32), ("syrk_splits", ctypes.c_int32),
                ("moment_density", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("width", ctypes.c_int32), ("msp", ctypes.c_int32), ("Mr", ctypes.c_int32),
                ("L1", ctypes.c_int32), ("L2", ctypes.c_int32), ("fused", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("beta", ctypes.c_double), ("tol", ctypes.c_double),
                ("est_err", ctypes.c_double)]


_lib = None


def lib():
    """Load libmm.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmm.so is not built; run `python -m paper_2003_02842_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        L.mm_plan_query.argtypes = [i32, i32, f64, i32, P, P]
        L.mm_nufft1_workspace_size.argtypes = [i32, i32, i32, f64, i32, P, ctypes.POINTER(sz)]
        L.mm_nufft1.argtypes = [i32, P, P, P, i32, f64, f64, i32, i32, f64, i32, P, P, i64, P, sz, i32, P]
        L.mm_cov_workspace_size.argtypes = [i32, i32, i32, i32, i32, P, ctypes.POINTER(sz)]
        L.mm_cov.argtypes = [i32, i32, P, i64, P, i32, i32, i32, P, P, P, P, sz, P]
        L.mm_estimate_workspace_size.argtypes = [i32, i32, P, i32, i32, f64, i32, P, ctypes.POINTER(sz)]
        L.mm_estimate.argtypes = [i32, i32, P, P, P, i32, f64, f64, P, i32, i32, i32, f64, i32, P, P, i64, P, P, P,
                                  sz, i32, P]
        L.mm_estimate_noalloc.argtypes = [i32, i32, P, P, P, i32, f64, f64, P, i32, i32, i32, f64, i32, P, P, i64,
                                          P, P, P]
        L.mm_graph_cache_clear.argtypes = []
        L.mm_snap_times.argtypes = [i64, P, f64, f64, i64, P, P]
        L.mm_cov_pairwise_workspace_size.argtypes = [i32, i32, P, i32, ctypes.POINTER(sz)]
        L.mm_cov_pairwise.argtypes = [i32, i32, P, i64, P, i32, i32, P, P, P, sz, P]
        L.mm_matrix_to_csr_workspace_size.argtypes = [i64, i32, ctypes.POINTER(sz)]
        L.mm_matrix_to_csr.argtypes = [i64, i32, P, P, i64, P, P, P, i32, i64, P, P, sz, P, P]
        L.mm_status_string.argtypes = [i32]
        L.mm_status_string.restype = ctypes.c_char_p
        L.mm_profile_enable.argtypes = [i32]
        L.mm_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(f64), ctypes.POINTER(i64)]
        for name in EXPORTED:
            if name != "mm_status_string":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _status_text(s: int) -> str:
    try:
        return lib().mm_status_string(int(s)).decode()
    except Exception:
        return "status %d" % s


def _check(status: int, where: str):
    if status != MM_OK:
        raise MMError(status, where)


def _enum(value, table, what):
    if isinstance(value, str):
        key = value.lower()
        if key not in table:
            raise ValueError("unknown %s %r" % (what, value))
        return table[key]
    return int(value)


def _tuning(tune):
    if tune is None:
        return None
    if isinstance(tune, Tuning):
        return tune
    t = Tuning()
    for k, v in dict(tune).items():
        setattr(t, k, v)
    return t


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def plan_query(N: int, kernel="es", tol: float = 1e-12, prec="fp64", tune=None) -> dict:
    info = PlanInfo()
    t = _tuning(tune)
    st = lib().mm_plan_query(int(N), _enum(kernel, _KERNELS, "kernel"), float(tol), _enum(prec, _PRECS, "precision"),
                             ctypes.byref(t) if t is not None else None, ctypes.byref(info))
    _check(st, "mm_plan_query")
    return {f: getattr(info, f) for f, _ in PlanInfo._fields_}


def nufft1_workspace_size(S: int, N: int, kernel="es", tol=1e-12, prec="fp64", tune=None) -> int:
    out = ctypes.c_size_t(0)
    t = _tuning(tune)
    st = lib().mm_nufft1_workspace_size(int(S), int(N), _enum(kernel, _KERNELS, "kernel"), float(tol),
                                        _enum(prec, _PRECS, "precision"), ctypes.byref(t) if t is not None else None,
                                        ctypes.byref(out))
    _check(st, "mm_nufft1_workspace_size")
    return int(out.value)


def _workspace(nbytes: int, device):
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def nufft1(offsets: torch.Tensor, t: torch.Tensor, dp: torch.Tensor, t0: float, T: float, N: int, kernel="es",
           tol: float = 1e-12, prec="fp64", tune=None, validate: bool = False, out: torch.Tensor = None,
           ws: torch.Tensor = None) -> torch.Tensor:
    """Coefficients c_k, k = 0..N, of every CSR series: (S, N+1) complex128
    (prec "fp64") or complex64 (prec "mixed")."""
    p = _enum(prec, _PRECS, "precision")
    if not (offsets.is_cuda and t.is_cuda and dp.is_cuda):
        raise ValueError("offsets, t and dp must be device tensors")
    if offsets.dtype != torch.int64 or t.dtype != torch.float64 or dp.dtype not in (torch.float32, torch.float64):
        raise TypeError("offsets int64, t float64, dp float32/float64 expected")
    offsets, t, dp = offsets.contiguous(), t.contiguous(), dp.contiguous()
    S = offsets.numel() - 1
    cdt = torch.complex64 if p == MIXED else torch.complex128
    if out is None:
        out = torch.empty((S, N + 1), dtype=cdt, device=t.device)
    if out.dtype != cdt or out.dim() != 2 or out.shape[0] != S or out.stride(1) != 1:
        raise ValueError("out must be (S, ldc>=N+1) %s with unit column stride" % cdt)
    need = nufft1_workspace_size(S, N, kernel, tol, prec, tune)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, t.device)
    tt = _tuning(tune)
    st = lib().mm_nufft1(S, _ptr(offsets), _ptr(t), _ptr(dp), int(dp.dtype == torch.float64), float(t0), float(T),
                         int(N), _enum(kernel, _KERNELS, "kernel"), float(tol), p,
                         ctypes.byref(tt) if tt is not None else None, _ptr(out), out.stride(0), _ptr(ws),
                         ws.numel() if ws is not None else 0, int(bool(validate)), _stream())
    _check(st, "mm_nufft1")
    return out


def cov_workspace_size(G: int, D: int, Nmax: int, nN: int, prec="fp64", tune=None) -> int:
    out = ctypes.c_size_t(0)
    t = _tuning(tune)
    _check(lib().mm_cov_workspace_size(int(G), int(D), int(Nmax), int(nN), _enum(prec, _PRECS, "precision"),
                                       ctypes.byref(t) if t is not None else None, ctypes.byref(out)),
           "mm_cov_workspace_size")
    return int(out.value)


def cov(coef: torch.Tensor, G: int, D: int, Ns, basis="dirichlet", correlation: bool = True, ws: torch.Tensor = None,
        tune=None):
    """Sigma (and R) of shape (len(Ns), G, D, D) from (G*D, >=max(Ns)+1) coefficients;
    ``tune`` may set the contraction's tile (syrk_tile) and k-split (syrk_splits)."""
    if coef.dtype == torch.complex64:
        p, rdt = MIXED, torch.float32
    elif coef.dtype == torch.complex128:
        p, rdt = PLAIN_FP64, torch.float64
    else:
        raise TypeError("coef must be complex64 (mixed) or complex128 (fp64)")
    if not coef.is_cuda or coef.dim() != 2 or coef.stride(1) != 1 or coef.shape[0] != G * D:
        raise ValueError("coef must be a (G*D, ldc) device tensor with unit column stride")
    Ns = [int(n) for n in Ns]
    arr = (ctypes.c_int32 * len(Ns))(*Ns)
    covt = torch.empty((len(Ns), G, D, D), dtype=rdt, device=coef.device)
    corrt = torch.empty_like(covt) if correlation else None
    need = cov_workspace_size(G, D, max(Ns), len(Ns), "mixed" if p == MIXED else "fp64", tune)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, coef.device)
    tt = _tuning(tune)
    st = lib().mm_cov(int(G), int(D), _ptr(coef), coef.stride(0), arr, len(Ns), _enum(basis, _BASES, "basis"), p,
                      ctypes.byref(tt) if tt is not None else None, _ptr(covt), _ptr(corrt), _ptr(ws),
                      ws.numel() if ws is not None else 0, _stream())
    _check(st, "mm_cov")
    return covt, corrt


def estimate_workspace_size(G: int, D: int, Ns, kernel="es", tol: float = 1e-12, prec="fp64", tune=None) -> int:
    Ns = [int(n) for n in Ns]
    arr = (ctypes.c_int32 * len(Ns))(*Ns)
    out = ctypes.c_size_t(0)
    t = _tuning(tune)
    _check(lib().mm_estimate_workspace_size(int(G), int(D), arr, len(Ns), _enum(kernel, _KERNELS, "kernel"),
                                            float(tol), _enum(prec, _PRECS, "precision"),
                                            ctypes.byref(t) if t is not None else None, ctypes.byref(out)),
           "mm_estimate_workspace_size")
    return int(out.value)


_graph_streams = {}


def estimate(offsets: torch.Tensor, t: torch.Tensor, dp: torch.Tensor, t0: float, T: float, G: int, D: int, Ns,
             basis="dirichlet", kernel="es", tol: float = 1e-12, prec="fp64", tune=None, use_graph: bool = False,
             coef: torch.Tensor = None, correlation: bool = True, ws: torch.Tensor = None,
             out=None):
    """Both stages in one library call (mm_estimate): Sigma (and R) of shape
    (len(Ns), G, D, D) for G groups of D consecutive CSR series.  With
    ``use_graph`` the launch sequence is recorded once into a HIP graph and
    replayed by later calls with the same tensors; on torch's default stream the
    call runs on a side stream ordered after and before the current one.
    ``out`` = (cov, corr) reuses output tensors (needed for replays to hit the
    same graph)."""
    p = _enum(prec, _PRECS, "precision")
    if not (offsets.is_cuda and t.is_cuda and dp.is_cuda):
        raise ValueError("offsets, t and dp must be device tensors")
    if offsets.dtype != torch.int64 or t.dtype != torch.float64 or dp.dtype not in (torch.float32, torch.float64):
        raise TypeError("offsets int64, t float64, dp float32/float64 expected")
    if not (offsets.is_contiguous() and t.is_contiguous() and dp.is_contiguous()):
        raise ValueError("offsets, t and dp must be contiguous")
    Ns = [int(n) for n in Ns]
    arr = (ctypes.c_int32 * len(Ns))(*Ns)
    rdt = torch.float32 if p == MIXED else torch.float64
    if out is None:
        covt = torch.empty((len(Ns), G, D, D), dtype=rdt, device=t.device)
        corrt = torch.empty_like(covt) if correlation else None
    else:
        covt, corrt = out
    need = estimate_workspace_size(G, D, Ns, kernel, tol, prec, tune)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, t.device)
    tt = _tuning(tune)
    ldc = coef.stride(0) if coef is not None else 0
    args = [int(G), int(D), _ptr(offsets), _ptr(t), _ptr(dp), int(dp.dtype == torch.float64), float(t0), float(T),
            arr, len(Ns), _enum(basis, _BASES, "basis"), _enum(kernel, _KERNELS, "kernel"), float(tol), p,
            ctypes.byref(tt) if tt is not None else None, _ptr(coef), ldc, _ptr(covt), _ptr(corrt), _ptr(ws),
            ws.numel(), int(bool(use_graph))]
    cur = torch.cuda.current_stream()
    if use_graph and cur.cuda_stream == 0:
        side = _graph_streams.get(t.device)
        if side is None:
            side = _graph_streams[t.device] = torch.cuda.Stream(device=t.device)
        side.wait_stream(cur)
        st = lib().mm_estimate(*args, ctypes.c_void_p(side.cuda_stream))
        cur.wait_stream(side)
    else:
        st = lib().mm_estimate(*args, ctypes.c_void_p(cur.cuda_stream))
    _check(st, "mm_estimate")
    return covt, corrt, ws


SCRATCH_BYTES = 64 << 20   # MM_SCRATCH_BYTES


def estimate_noalloc(offsets: torch.Tensor, t: torch.Tensor, dp: torch.Tensor, t0: float, T: float, G: int, D: int,
                     Ns, basis="dirichlet", kernel="es", tol: float = 1e-12, prec="fp64", tune=None,
                     coef: torch.Tensor = None, out=None):
    """mm_estimate_noalloc: both stages with the library's fixed device scratch
    (MM_SCRATCH_BYTES per GPU) instead of a workspace argument.  ``out`` =
    (cov, corr) are written when given (no allocation at all here then), else
    allocated.  Returns (cov, corr)."""
    p = _enum(prec, _PRECS, "precision")
    if not (offsets.is_cuda and t.is_cuda and dp.is_cuda):
        raise ValueError("offsets, t and dp must be device tensors")
    if offsets.dtype != torch.int64 or t.dtype != torch.float64 or dp.dtype not in (torch.float32, torch.float64):
        raise TypeError("offsets int64, t float64, dp float32/float64 expected")
    if not (offsets.is_contiguous() and t.is_contiguous() and dp.is_contiguous()):
        raise ValueError("offsets, t and dp must be contiguous")
    Ns = [int(n) for n in Ns]
    arr = (ctypes.c_int32 * len(Ns))(*Ns)
    rdt = torch.float32 if p == MIXED else torch.float64
    if out is None:
        covt = torch.empty((len(Ns), G, D, D), dtype=rdt, device=t.device)
        corrt = torch.empty_like(covt)
    else:
        covt, corrt = out
    tt = _tuning(tune)
    ldc = coef.stride(0) if coef is not None else 0
    st = lib().mm_estimate_noalloc(int(G), int(D), _ptr(offsets), _ptr(t), _ptr(dp), int(dp.dtype == torch.float64),
                                   float(t0), float(T), arr, len(Ns), _enum(basis, _BASES, "basis"),
                                   _enum(kernel, _KERNELS, "kernel"), float(tol), p,
                                   ctypes.byref(tt) if tt is not None else None, _ptr(coef), ldc, _ptr(covt),
                                   _ptr(corrt), _stream())
    _check(st, "mm_estimate_noalloc")
    return covt, corrt


def graph_cache_clear():
    _check(lib().mm_graph_cache_clear(), "mm_graph_cache_clear")


def profile_enable(on: bool = True):
    _check(lib().mm_profile_enable(int(bool(on))), "mm_profile_enable")


def profile_reset():
    _check(lib().mm_profile_reset(), "mm_profile_reset")


def profile_read(name=None):
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(lib().mm_profile_read(name.encode() if name else None, ctypes.byref(ms), ctypes.byref(n)),
           "mm_profile_read")
    return float(ms.value), int(n.value)


def matrix_to_csr(P: torch.Tensor, T: torch.Tensor, dp_dtype=torch.float32, ws: torch.Tensor = None):
    """The MM algorithm's input form -- (n, D) device tensors of prices and
    times, NaN where an asset has no observation -- to CSR returns
    (mm_matrix_to_csr).  Returns (offsets, t, dp, nyq, info) where info holds
    E, the Nyquist cutoff N = min_i N_i and the window (t0, T)."""
    if not (P.is_cuda and T.is_cuda) or P.dtype != torch.float64 or T.dtype != torch.float64:
        raise TypeError("P and T must be float64 device tensors")
    if P.shape != T.shape or P.dim() != 2:
        raise ValueError("P and T must have the same (n, D) shape")
    n, D = P.shape
    Pc = P.t().contiguous()   # column-major n x D: asset i contiguous
    Tc = T.t().contiguous()
    dev = P.device
    need = ctypes.c_size_t(0)
    _check(lib().mm_matrix_to_csr_workspace_size(n, D, ctypes.byref(need)), "mm_matrix_to_csr_workspace_size")
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(need.value, dtype=torch.uint8, device=dev)
    cap = n * D
    offsets = torch.empty(D + 1, dtype=torch.int64, device=dev)
    t = torch.empty(cap, dtype=torch.float64, device=dev)
    dp = torch.empty(cap, dtype=dp_dtype, device=dev)
    nyq = torch.empty(D, dtype=torch.int32, device=dev)
    info = CsrInfo()
    st = lib().mm_matrix_to_csr(n, D, _ptr(Pc), _ptr(Tc), n, _ptr(offsets), _ptr(t), _ptr(dp),
                                int(dp_dtype == torch.float64), cap, _ptr(nyq), _ptr(ws), ws.numel(),
                                ctypes.byref(info), _stream())
    _check(st, "mm_matrix_to_csr")
    E = int(info.E)
    return offsets, t[:E], dp[:E], nyq, {"E": E, "N": int(info.N), "t0": info.t0, "T": info.T}


def snap_times(t: torch.Tensor, t0: float, T: float, Nstar: int) -> torch.Tensor:
    """Times moved to the nearest of Nstar equally spaced points of [t0, T)
    (mm_snap_times): the zero-padded FFT method as a negative control."""
    if not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("t must be a float64 device tensor")
    t = t.contiguous()
    out = torch.empty_like(t)
    _check(lib().mm_snap_times(t.numel(), _ptr(t), float(t0), float(T), int(Nstar), _ptr(out), _stream()),
           "mm_snap_times")
    return out


def cov_pairwise(coef: torch.Tensor, G: int, D: int, Ni, basis="dirichlet", correlation: bool = True,
                 ws: torch.Tensor = None):
    """Pairwise estimates at N_ij = min(N_i, N_j) (mm_cov_pairwise): (G, D, D)
    covariance and correlation."""
    if coef.dtype == torch.complex64:
        p, rdt = MIXED, torch.float32
    elif coef.dtype == torch.complex128:
        p, rdt = PLAIN_FP64, torch.float64
    else:
        raise TypeError("coef must be complex64 (mixed) or complex128 (fp64)")
    if not coef.is_cuda or coef.dim() != 2 or coef.stride(1) != 1 or coef.shape[0] != G * D:
        raise ValueError("coef must be a (G*D, ldc) device tensor with unit column stride")
    Ni = [int(n) for n in Ni]
    if len(Ni) != D:
        raise ValueError("Ni must hold one cutoff per asset")
    arr = (ctypes.c_int32 * D)(*Ni)
    need = ctypes.c_size_t(0)
    _check(lib().mm_cov_pairwise_workspace_size(int(G), int(D), arr, p, ctypes.byref(need)),
           "mm_cov_pairwise_workspace_size")
    if ws is None or ws.numel() < need.value:
        ws = _workspace(need.value, coef.device)
    covt = torch.empty((G, D, D), dtype=rdt, device=coef.device)
    corrt = torch.empty_like(covt) if correlation else None
    _check(lib().mm_cov_pairwise(int(G), int(D), _ptr(coef), coef.stride(0), arr, _enum(basis, _BASES, "basis"), p,
                                 _ptr(covt), _ptr(corrt), _ptr(ws), ws.numel(), _stream()), "mm_cov_pairwise")
    return covt, corrt
