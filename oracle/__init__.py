"""Python access to the plain FP64 CPU oracle (``mm_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The GPU library never imports it.

The oracle evaluates the paper's definitions directly (Sec. 2.1-2.2):
coefficients c_k = (1/2pi) sum_h delta_h exp(-i k tilde t_h) (equation
F(dp_i)(k)), the Dirichlet/Fejer estimators (Eqs. Der:2, Der:3) and the
correlation step of the MM algorithm.  See ``mm_oracle.c`` for the arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DIRICHLET, FEJER = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.orc_coeffs.argtypes = [i64, P, P, f64, f64, i64, i64, P]
        L.orc_coeffs_at.argtypes = [i64, P, P, f64, f64, P, i64, P]
        L.orc_coeffs_batch.argtypes = [i32, P, P, P, f64, f64, i32, P, i64]
        L.orc_cov_full.argtypes = [i32, i32, P, i64, i32, i32, P, P, P]
        L.orc_cov.argtypes = [i32, i32, P, i64, P, i32, i32, P, P]
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().orc_threads())


def _np(x, dtype):
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(x, dtype=dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def coeffs(t, dp, t0: float, T: float, klo: int, khi: int) -> np.ndarray:
    """c_k for k = klo..khi of one series (complex128)."""
    t = _np(t, np.float64)
    dp = _np(dp, np.float64)
    out = np.zeros(2 * (khi - klo + 1), dtype=np.float64)
    lib().orc_coeffs(t.size, _p(t), _p(dp), t0, T, klo, khi, _p(out))
    return out.view(np.complex128)


def coeffs_at(t, dp, t0: float, T: float, ks) -> np.ndarray:
    """c_k of one series at the listed frequencies ks (complex128, same order)."""
    t = _np(t, np.float64)
    dp = _np(dp, np.float64)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    out = np.zeros(2 * ks.size, dtype=np.float64)
    lib().orc_coeffs_at(t.size, _p(t), _p(dp), t0, T, _p(ks), ks.size, _p(out))
    return out.view(np.complex128)


def coeffs_batch(offsets, t, dp, t0: float, T: float, N: int) -> np.ndarray:
    """(S, N+1) complex128 coefficients, k = 0..N, of CSR series."""
    offsets = _np(offsets, np.int64)
    t = _np(t, np.float64)
    dp = _np(dp, np.float64)
    S = offsets.size - 1
    out = np.zeros((S, 2 * (N + 1)), dtype=np.float64)
    lib().orc_coeffs_batch(S, _p(offsets), _p(t), _p(dp), t0, T, N, _p(out), N + 1)
    return out.view(np.complex128)


def cov(coef: np.ndarray, G: int, D: int, Ns, basis: int):
    """Sigma and R for each cutoff in Ns from k = 0..max(Ns) coefficients.
    Returns arrays of shape (len(Ns), G, D, D)."""
    coef = np.ascontiguousarray(coef, dtype=np.complex128)
    Ns = np.ascontiguousarray(list(Ns), dtype=np.int32)
    assert coef.shape[0] == G * D and coef.shape[1] >= int(Ns.max()) + 1
    c = np.ascontiguousarray(coef.view(np.float64))
    out = np.zeros((Ns.size, G, D, D))
    corr = np.zeros_like(out)
    lib().orc_cov(G, D, _p(c), coef.shape[1], _p(Ns), Ns.size, basis, _p(out), _p(corr))
    return out, corr


def cov_full(coef_full: np.ndarray, G: int, D: int, N: int, basis: int):
    """Complex Sigma (and R from its real part) from coefficients s = -N..N."""
    coef_full = np.ascontiguousarray(coef_full, dtype=np.complex128)
    assert coef_full.shape == (G * D, 2 * N + 1)
    c = np.ascontiguousarray(coef_full.view(np.float64))
    re = np.zeros((G, D, D))
    im = np.zeros_like(re)
    corr = np.zeros_like(re)
    lib().orc_cov_full(G, D, _p(c), 2 * N + 1, N, basis, _p(re), _p(im), _p(corr))
    return re + 1j * im, corr


def estimate(w, Ns=None, basis: int = DIRICHLET):
    """Coefficients and (Sigma, R) of a ``synth.Workload`` for cutoffs Ns."""
    Ns = list(w.Ns if Ns is None else Ns)
    coef = coeffs_batch(w.offsets, w.t, w.dp, w.t0, w.T, max(Ns))
    S, R = cov(coef, w.G, w.D, Ns, basis)
    return coef, S, R


INT32_MAX = 2 ** 31 - 1


def matrix_to_csr(P, T):
    """The MM algorithm's input form to CSR returns (steps F.1-F.3), the window of
    the time-rescaling algorithm and the cutoffs of the Nyquist-frequency
    algorithm, in plain numpy.

    P, T: (n, D) arrays, NaN where asset i has no observation; an observation
    counts when both entries are finite.  Window: min and max of all counted
    times.  Asset i: its counted times in row order, log prices, returns
    log p_{h+1} - log p_h at time t_h; dt_i = smallest gap between consecutive
    times; N_i = floor((t_max - t_min) / (2 dt_i)) (the algorithm's
    floor(N_0/2) with N_0 = 2 pi / dt on times rescaled to [0, 2 pi]), capped
    at 2^31 - 1; N = min_i N_i.  Returns (offsets, t, dp, nyq, N, (t0, T))."""
    P = np.asarray(P, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n, D = P.shape
    valid = np.isfinite(P) & np.isfinite(T)
    t0, t1 = float(T[valid].min()), float(T[valid].max())
    offsets, ts, dps, nyq = [0], [], [], []
    for i in range(D):
        tv = T[valid[:, i], i]
        lp = np.log(P[valid[:, i], i])
        if tv.size >= 2:
            ts.append(tv[:-1])
            dps.append(lp[1:] - lp[:-1])
            gaps = tv[1:] - tv[:-1]
            # cutoffs are int32 at the library boundary: larger values are capped there
            nyq.append(min(int(np.floor((t1 - t0) / (2.0 * gaps.min()))), INT32_MAX))
        else:
            nyq.append(INT32_MAX)
        offsets.append(offsets[-1] + max(tv.size - 1, 0))
    t = np.concatenate(ts) if ts else np.zeros(0)
    dp = np.concatenate(dps) if dps else np.zeros(0)
    return np.array(offsets, dtype=np.int64), t, dp, np.array(nyq, dtype=np.int64), min(nyq), (t0, t1)


def snap_times(t, t0: float, T: float, Nstar: int) -> np.ndarray:
    """The zero-padded FFT method's grid assignment (appendix algorithm): each time
    moves to the nearest of Nstar equally spaced points of [t0, T), the last
    point wrapping to t0 (rounding half to even, like the C library's rint)."""
    t = _np(t, np.float64)
    span = T - t0
    l = np.rint(((t - t0) / span) * float(Nstar)).astype(np.int64)
    l[l >= Nstar] -= Nstar
    return t0 + span * (l.astype(np.float64) / float(Nstar))


def cov_pairwise(coef: np.ndarray, G: int, D: int, Ni, basis: int):
    """Pairwise estimates (Sec. 3): entry (i, j) is the 2 x 2 estimate of the pair
    at N_ij = min(N_i, N_j); R_ij from that 2 x 2 estimate.  Shapes (G, D, D)."""
    Ni = [int(n) for n in Ni]
    cov_out = np.zeros((G, D, D))
    corr_out = np.zeros((G, D, D))
    for g in range(G):
        for i in range(D):
            for j in range(D):
                N = min(Ni[i], Ni[j])
                rows = np.ascontiguousarray(coef[[g * D + i, g * D + j], :N + 1])
                S2, R2 = cov(rows, 1, 2, [N], basis)
                cov_out[g, i, j] = S2[0, 0, 0, 1] if i != j else S2[0, 0, 0, 0]
                corr_out[g, i, j] = R2[0, 0, 0, 1] if i != j else R2[0, 0, 0, 0]
    return cov_out, corr_out
