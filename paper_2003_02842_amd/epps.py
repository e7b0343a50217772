"""Time scales of the estimator and the Epps-effect model (Sec. 4 of the paper).

A cutoff N examines the sampling interval dt through Eq. Der:22,
N = floor((T/dt - 1)/2), so one NUFFT at the largest N and one sweep of the
contraction give the correlation at every time scale (``sweep``).  Eq. Der:21
is the Epps curve of two assets sampled by Poisson arrivals of intensity lam,
rho(dt) = c (1 + (exp(-lam dt) - 1)/(lam dt)); ``fit_epps`` fits c (and, if
asked, lam) to measured correlations by least squares.

The sweep runs on the GPU through the C ABI (mm_estimate); the fit is a host
computation on its output.
"""
from __future__ import annotations

import math

import numpy as np


def cutoff_for_interval(T: float, dt: float) -> int:
    """Eq. Der:22: N = floor((T/dt - 1)/2)."""
    return int(math.floor(0.5 * (T / dt - 1.0)))


def interval_for_cutoff(T: float, N: int) -> float:
    """The sampling interval a cutoff examines, dt = T/(2N + 1) (Sec. 4)."""
    return T / (2.0 * N + 1.0)


def epps_model(dt, c: float, lam: float):
    """Eq. Der:21: c (1 + (exp(-lam dt) - 1)/(lam dt))."""
    x = lam * np.asarray(dt, dtype=np.float64)
    return c * (1.0 + np.expm1(-x) / x)


def _fit_c(dt, rho, lam):
    g = epps_model(dt, 1.0, lam)
    c = float(np.dot(g, rho) / np.dot(g, g))
    return c, float(np.sum((rho - c * g) ** 2))


def fit_epps(dt, rho, lam: float = None):
    """Least-squares fit of Eq. Der:21 to correlations rho measured at intervals
    dt.  With lam given only c is fitted (closed form, the model is linear in c);
    otherwise lam is found by golden-section search on log(lam) with c fitted in
    closed form at every step.  Returns (c, lam, residual sum of squares)."""
    dt = np.asarray(dt, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    if lam is not None:
        c, rss = _fit_c(dt, rho, lam)
        return c, float(lam), rss
    lo, hi = math.log(1e-3 / dt.max()), math.log(1e3 / dt.min())
    phi = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    x1, x2 = b - phi * (b - a), a + phi * (b - a)
    f1, f2 = _fit_c(dt, rho, math.exp(x1))[1], _fit_c(dt, rho, math.exp(x2))[1]
    for _ in range(200):
        if f1 < f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - phi * (b - a)
            f1 = _fit_c(dt, rho, math.exp(x1))[1]
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + phi * (b - a)
            f2 = _fit_c(dt, rho, math.exp(x2))[1]
        if b - a < 1e-12:
            break
    lam = math.exp(0.5 * (a + b))
    c, rss = _fit_c(dt, rho, lam)
    return c, lam, rss


def sweep(offsets, t, dp, t0: float, T: float, G: int, D: int, dts, basis="dirichlet", kernel="es",
          tol: float = 1e-6, prec="mixed"):
    """Correlations at the sampling intervals dts (same time unit as t) for G
    groups of D series: one NUFFT at the largest cutoff, one contraction sweep.
    Returns (Ns, R) with R of shape (len(Ns), G, D, D); duplicate cutoffs are
    merged (Ns sorted ascending)."""
    from paper_2003_02842_amd import mm
    span = T - t0
    Ns = sorted({max(1, cutoff_for_interval(span, dt)) for dt in dts})
    _, R, _ = mm.estimate(offsets, t, dp, t0, T, G, D, Ns, basis, kernel, tol, prec)
    return Ns, R
