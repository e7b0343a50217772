"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars: FP64 path within 1e-11 relative Frobenius of the oracle for Sigma and R
(and per-series coefficient l2 error within the requested tolerance); mixed
path (FP32 spreading/FFT, split-BF16 MFMA contraction) within 1e-5.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2003_02842_amd import synth
from tests.helpers import need_gpu, relfro, series_rel_l2

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-11
MIXED_BAR = 1e-5


@pytest.fixture(scope="module")
def mm():
    need_gpu()
    from paper_2003_02842_amd import mm as m
    return m


def oracle_coef(w, N):
    return oracle.coeffs_batch(w.offsets, w.t, w.dp, w.t0, w.T, N)


def gpu_coef(mm, w, N, kernel, tol, prec, tune=None):
    wd = w.to("cuda")
    c = mm.nufft1(wd.offsets, wd.t, wd.dp, w.t0, w.T, N, kernel, tol, prec, tune)
    torch.cuda.synchronize()
    return c


# ------------------------------------------------------------------ single jump
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
@pytest.mark.parametrize("kernel", ["es", "kb", "g"])
@pytest.mark.parametrize("u", [0.0, 0.25, 0.5 - 2 ** -30, 1.0 - 2 ** -40, 1.0, 37.0 / 1350.0])
def test_single_jump(mm, prec, tol, kernel, u):
    N = 333
    w = synth.single_jump(u, 0.7, dp_dtype=torch.float64 if prec == "fp64" else torch.float32)
    c = gpu_coef(mm, w, N, kernel, tol, prec).cpu().numpy()
    ref = oracle_coef(w, N)
    err = series_rel_l2(c, ref)[0]
    assert err <= tol, err


# ------------------------------------------- tiny synchronous bivariate, FP64 path
@pytest.mark.parametrize("kernel", ["es", "kb", "g"])
def test_bivariate_sync_fp64(mm, kernel):
    w = synth.bivariate_sync(n=10_000)
    N = w.Ns[0]
    c = gpu_coef(mm, w, N, kernel, 1e-12, "fp64")
    ref = oracle_coef(w, N)
    assert series_rel_l2(c, ref).max() <= 1e-12
    for basis, b in (("dirichlet", oracle.DIRICHLET), ("fejer", oracle.FEJER)):
        S, R = mm.cov(c, 1, 2, [N], basis)
        So, Ro = oracle.cov(ref, 1, 2, [N], b)
        assert relfro(S.cpu().numpy(), So) <= FP64_BAR
        assert relfro(R.cpu().numpy(), Ro) <= FP64_BAR


# --------------------------------------------- asynchronous bivariate, N sweep, mixed
@pytest.mark.parametrize("kernel", ["es", "kb", "g"])
@pytest.mark.parametrize("basis", ["dirichlet", "fejer"])
def test_bivariate_async_sweep_mixed(mm, kernel, basis):
    w = synth.bivariate_async()
    assert len(w.Ns) >= 30
    Nmax = max(w.Ns)
    c = gpu_coef(mm, w, Nmax, kernel, 1e-6, "mixed")
    S, R = mm.cov(c, 1, 2, w.Ns, basis)
    ref = oracle_coef(w, Nmax)
    So, Ro = oracle.cov(ref, 1, 2, w.Ns, oracle.DIRICHLET if basis == "dirichlet" else oracle.FEJER)
    S, R = S.cpu().numpy(), R.cpu().numpy()
    for q in range(len(w.Ns)):
        assert relfro(S[q], So[q]) <= MIXED_BAR, (w.Ns[q], relfro(S[q], So[q]))
        assert relfro(R[q], Ro[q]) <= MIXED_BAR, (w.Ns[q], relfro(R[q], Ro[q]))


# ------------------------------------------ ragged series, empty series, many tiles
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
@pytest.mark.parametrize("tile", [1024, 4096, 0])
@pytest.mark.parametrize("kernel", ["es", "g", "kb"])
def test_ragged_many_tiles(mm, prec, tol, tile, kernel):
    """Uneven and empty series over a grid of several tiles (Mr = 12150); one
    dense series (about 4 events per cell) makes tiles span several LDS chunks."""
    w = synth.random_events(9, 0, 3000, seed=123, dp_dtype=torch.float64 if prec == "fp64" else torch.float32)
    dense = synth.random_events(1, 50_000, 50_000, seed=7, dp_dtype=w.dp.dtype)
    w = synth.Workload("ragged", torch.cat([w.offsets, w.offsets[-1] + dense.offsets[1:]]),
                       torch.cat([w.t, dense.t]), torch.cat([w.dp, dense.dp]), 0.0, 1.0, 1, 10, [1], 0, {})
    counts = (w.offsets[1:] - w.offsets[:-1]).tolist()
    N = 3000
    tune = {"tile": tile} if tile else None
    c = gpu_coef(mm, w, N, kernel, tol, prec, tune)
    ref = oracle_coef(w, N)
    err = series_rel_l2(c, ref)
    bar = tol
    for s, n in enumerate(counts):
        if n == 0:
            assert np.all(c[s].cpu().numpy() == 0)
        else:
            assert err[s] <= bar, (s, n, err[s])
    S, R = mm.cov(c, 1, 10, [N, 17], "fejer")
    So, Ro = oracle.cov(ref, 1, 10, [N, 17], oracle.FEJER)
    bar2 = FP64_BAR if prec == "fp64" else MIXED_BAR
    assert relfro(S.cpu().numpy(), So) <= bar2
    assert relfro(R.cpu().numpy(), Ro) <= bar2


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_edge_times(mm, prec, tol):
    """Events exactly at t0, exactly at T (the same point as t0), on grid nodes,
    and duplicated timestamps."""
    N = 40
    Mr = mm.plan_query(N, "es", tol, prec)["Mr"]
    T = 3.0
    t = torch.tensor([0.0, 0.0, T * 5 / Mr, T * 0.5, T * (Mr - 1) / Mr, T], dtype=torch.float64)
    dp = torch.tensor([0.1, -0.2, 0.3, 0.05, -0.4, 0.25], dtype=torch.float64 if prec == "fp64" else torch.float32)
    w = synth.Workload("edge", torch.tensor([0, 6], dtype=torch.int64), t, dp, 0.0, T, 1, 1, [N], 0, {})
    c = gpu_coef(mm, w, N, "es", tol, prec)
    ref = oracle_coef(w, N)
    assert series_rel_l2(c, ref)[0] <= tol


def test_validate_rejects_bad_data(mm):
    base = synth.random_events(3, 5, 20, seed=4)
    good = base.to("cuda")
    mm.nufft1(good.offsets, good.t, good.dp, 0.0, 1.0, 10, "es", 1e-6, "fp64", validate=True)
    bad_cases = []
    t = good.t.clone(); t[3], t[4] = t[4].item(), t[3].item() + 1e-9; bad_cases.append((t, good.dp))
    t = good.t.clone(); t[0] = 1.5; bad_cases.append((t, good.dp))
    d = good.dp.clone(); d[2] = float("nan"); bad_cases.append((good.t, d))
    t = good.t.clone(); t[1] = float("inf"); bad_cases.append((t, good.dp))
    for tt, dd in bad_cases:
        with pytest.raises(mm.MMError) as ei:
            mm.nufft1(good.offsets, tt, dd, 0.0, 1.0, 10, "es", 1e-6, "fp64", validate=True)
        assert ei.value.status == mm.MM_ERR_DATA


# ------------------------------------------- cross-section (MFMA contraction), reduced horizon
def test_cross_section_mfma(mm):
    w = synth.cross_section(D=100, T_sec=7200.0, N=5000, seed=99)
    N = 5000
    c = gpu_coef(mm, w, N, "es", 1e-6, "mixed")
    S, R = mm.cov(c, 1, 100, [N], "fejer")
    ref = oracle_coef(w, N)
    So, Ro = oracle.cov(ref, 1, 100, [N], oracle.FEJER)
    eS, eR = relfro(S.cpu().numpy(), So), relfro(R.cpu().numpy(), Ro)
    assert eS <= MIXED_BAR and eR <= MIXED_BAR, (eS, eR)
    # the same coefficients through the FP64 contraction
    c64 = gpu_coef(mm, w, N, "es", 1e-12, "fp64")
    S64, R64 = mm.cov(c64, 1, 100, [N], "fejer")
    assert relfro(S64.cpu().numpy(), So) <= FP64_BAR


# ----------------------------------------------- Monte Carlo replicates, reduced G
@pytest.mark.parametrize("basis", ["dirichlet", "fejer"])
def test_epps_replicates_sweep(mm, basis):
    w = synth.epps_replicates(G=12, seed=31)
    Nmax = max(w.Ns)
    c = gpu_coef(mm, w, Nmax, "es", 1e-6, "mixed")
    S, R = mm.cov(c, w.G, w.D, w.Ns, basis)
    ref = oracle_coef(w, Nmax)
    So, Ro = oracle.cov(ref, w.G, w.D, w.Ns, oracle.DIRICHLET if basis == "dirichlet" else oracle.FEJER)
    S, R = S.cpu().numpy(), R.cpu().numpy()
    for q in range(len(w.Ns)):
        for g in range(w.G):
            assert relfro(S[q, g], So[q, g]) <= MIXED_BAR
            assert relfro(R[q, g], Ro[q, g]) <= MIXED_BAR


# ---------------------------------------- both grid-FFT implementations agree
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
@pytest.mark.parametrize("N", [1, 2, 7, 100, 3000])
def test_generic_and_codelet_fft_paths(mm, prec, tol, N):
    """The register-codelet two-pass FFT and the generic in-LDS radix passes
    (mm_tuning.fft_generic = 1) both meet the bar against the oracle, from the
    smallest grids (Mr = 8) up to several thousand points."""
    w = synth.random_events(6, 0, 400, seed=31 + N, dp_dtype=torch.float64 if prec == "fp64" else torch.float32)
    ref = oracle_coef(w, N)
    bar = tol
    info = mm.plan_query(N, "es", tol, prec)
    for tune in (None, {"fft_generic": 1}):
        c = gpu_coef(mm, w, N, "es", tol, prec, tune)
        err = series_rel_l2(c, ref)
        counts = (w.offsets[1:] - w.offsets[:-1]).tolist()
        for s, n in enumerate(counts):
            if n:
                assert err[s] <= bar, (tune, info["Mr"], s, err[s])


# ------------------------------ both FP32 spreading evaluations meet the bar
@pytest.mark.parametrize("kernel", ["es", "g", "kb"])
@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("tol", [1e-6, 1e-3])
def test_spread_formula_and_polynomial_paths(mm, kernel, mode, tol):
    """mm_tuning.spread_direct = 1 (kernel formula at every pair) and 2 (per-tap
    polynomials evaluated once per event) on uneven series with a dense one."""
    w = synth.random_events(5, 0, 2000, seed=77, dp_dtype=torch.float32)
    dense = synth.random_events(1, 30_000, 30_000, seed=78, dp_dtype=torch.float32)
    w = synth.Workload("ragged", torch.cat([w.offsets, w.offsets[-1] + dense.offsets[1:]]),
                       torch.cat([w.t, dense.t]), torch.cat([w.dp, dense.dp]), 0.0, 1.0, 1, 6, [1], 0, {})
    N = 2500
    c = gpu_coef(mm, w, N, kernel, tol, "mixed", {"spread_direct": mode})
    ref = oracle_coef(w, N)
    err = series_rel_l2(c, ref)
    counts = (w.offsets[1:] - w.offsets[:-1]).tolist()
    for s, n in enumerate(counts):
        if n:
            assert err[s] <= tol, (s, n, err[s])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("sigma", [1.25, 1.55, 1.65, 2.5])
@pytest.mark.parametrize("kernel", ["es", "kb"])
def test_oversampling_factors(mm, prec, tol, mode, sigma, kernel):
    """Oversampling factors other than 2 (the planner widens the kernel until its
    error estimate, FP32 rounding included, is under tol: w = 9, 9, 7 for ES at
    tol 1e-6 and sigma = 1.55, 1.65, 2.5), both FP32 evaluations, uneven series
    with a dense one, Sigma/R at two cutoffs.  At sigma = 1.25 the deconvolution
    amplifies rounding (by ~40 at the band edge) past tol for every width, and
    the planner must say so; the per-pair formula, with more rounding than the
    polynomials, is refused at some of the other factors too."""
    N = 2700
    tune = {"sigma": sigma, "spread_direct": mode, "tile": 2048}
    if sigma == 1.25:
        with pytest.raises(mm.MMError, match="status 3"):
            mm.plan_query(N, kernel, tol, prec, tune)
        return
    try:
        info = mm.plan_query(N, kernel, tol, prec, tune)
    except mm.MMError as e:
        assert "status 3" in str(e) and prec == "mixed" and mode == 1, e
        return
    dt = torch.float64 if prec == "fp64" else torch.float32
    w = synth.random_events(7, 0, 2500, seed=91, dp_dtype=dt)
    dense = synth.random_events(1, 40_000, 40_000, seed=92, dp_dtype=dt)
    w = synth.Workload("ragged", torch.cat([w.offsets, w.offsets[-1] + dense.offsets[1:]]),
                       torch.cat([w.t, dense.t]), torch.cat([w.dp, dense.dp]), 0.0, 1.0, 1, 8, [1], 0, {})
    assert info["Mr"] >= sigma * (2 * N + 1)
    c = gpu_coef(mm, w, N, kernel, tol, prec, tune)
    ref = oracle_coef(w, N)
    err = series_rel_l2(c, ref)
    counts = (w.offsets[1:] - w.offsets[:-1]).tolist()
    bar = tol
    for s, n in enumerate(counts):
        if n:
            assert err[s] <= bar, (info["width"], info["Mr"], s, n, err[s])
    S, R = mm.cov(c, 1, 8, [N, 300], "fejer")
    So, Ro = oracle.cov(ref, 1, 8, [N, 300], oracle.FEJER)
    bar2 = FP64_BAR if prec == "fp64" else MIXED_BAR
    assert relfro(S.cpu().numpy(), So) <= bar2
    assert relfro(R.cpu().numpy(), Ro) <= bar2


@pytest.mark.parametrize("tile", [1024, 2048, 4096])
@pytest.mark.parametrize("per_cell", [0.02, 1.0, 4.0, 12.0, 80.0])
def test_polynomial_spreading_at_every_density(mm, tile, per_cell):
    """Densities from 0.02 to 80 events per grid cell: tiles holding a handful
    of events (one chunk, most cell pairs empty) up to tiles that take many LDS
    chunks, over several tiles and the periodic wrap."""
    N = 2100
    tune = {"spread_direct": 2, "tile": tile}
    plan = mm.plan_query(N, "es", 1e-6, "mixed", tune)
    n = max(1, int(per_cell * plan["Mr"]))
    w = synth.random_events(1, n, n, seed=int(per_cell * 100) + tile, dp_dtype=torch.float32)
    c = gpu_coef(mm, w, N, "es", 1e-6, "mixed", tune)
    ref = oracle_coef(w, N)
    err = series_rel_l2(c, ref)
    assert err[0] <= 1e-6, (n, plan["Mr"], err[0])


def _bursty_events(n_base, bursts, seed, dp_dtype=torch.float32):
    """One series on [0, 1): n_base uniform times plus dense bursts (lo, hi, n) of
    uniform times, so that one series has sparse tiles, dense tiles and tiles
    that straddle a burst's edge; bursts at 0 and 1 reach across the periodic wrap."""
    g = torch.Generator().manual_seed(seed)
    parts = [torch.rand(n_base, generator=g, dtype=torch.float64)]
    for lo, hi, n in bursts:
        parts.append(lo + (hi - lo) * torch.rand(n, generator=g, dtype=torch.float64))
    t, _ = torch.sort(torch.cat(parts))
    t = t.clamp(0.0, 1.0)
    dp = 1e-3 * torch.randn(t.numel(), generator=g, dtype=torch.float64)
    offs = torch.tensor([0, t.numel()], dtype=torch.int64)
    return synth.Workload("bursty", offs, t, dp.to(dp_dtype), 0.0, 1.0, 1, 1, [1], seed, {})


@pytest.mark.parametrize("per_cell", [0.5, 1.5, 6.4, 20.0])
@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_moment_and_tap_spreading_against_oracle(mm, per_cell, tile):
    """Dense tiles spread from per-cell moments (the default from one event per
    cell), per-event taps everywhere (moment_density -1), and moments for every
    tile holding an event (moment_density 1e-6): each within tol of the oracle."""
    N = 2100
    base = {"spread_direct": 2, "tile": tile}
    plan = mm.plan_query(N, "es", 1e-6, "mixed", base)
    n = max(1, int(per_cell * plan["Mr"]))
    w = synth.random_events(1, n, n, seed=int(per_cell * 10) + tile, dp_dtype=torch.float32)
    ref = oracle_coef(w, N)
    for md in (0.0, -1.0, 1e-6):
        c = gpu_coef(mm, w, N, "es", 1e-6, "mixed", dict(base, moment_density=md))
        err = series_rel_l2(c, ref)
        assert err[0] <= 1e-6, (md, n, plan["Mr"], err[0])


@pytest.mark.parametrize("kernel", ["es", "kb"])
@pytest.mark.parametrize("tile", [1024, 2048])
def test_moments_on_bursty_series_with_wrap(mm, kernel, tile):
    """A sparse background with bursts of 20-40 events per cell, two of them at
    the ends of the window (their kernels wrap around the periodic grid): the
    moment and tap kernels split one series' tiles between them with none left
    out or taken twice.  Within tol of the oracle, and bit-identical on a rerun."""
    N = 3000
    tune = {"spread_direct": 2, "tile": tile}
    plan = mm.plan_query(N, kernel, 1e-6, "mixed", tune)
    Mr = plan["Mr"]
    bursts = [(0.0, 0.004, int(40 * 0.004 * Mr)), (0.31, 0.33, int(20 * 0.02 * Mr)),
              (0.6, 0.6 + 1000 / Mr, int(30 * 1000)), (0.997, 1.0, int(30 * 0.003 * Mr))]
    w = _bursty_events(int(0.05 * Mr), bursts, seed=7 + tile)
    ref = oracle_coef(w, N)
    c1 = gpu_coef(mm, w, N, kernel, 1e-6, "mixed", tune)
    c2 = gpu_coef(mm, w, N, kernel, 1e-6, "mixed", tune)
    assert torch.equal(c1, c2)
    err = series_rel_l2(c1, ref)
    assert err[0] <= 1e-6, (kernel, tile, w.t.numel(), err[0])
    taps = gpu_coef(mm, w, N, kernel, 1e-6, "mixed", dict(tune, moment_density=-1.0))
    assert series_rel_l2(taps, ref)[0] <= 1e-6


@pytest.mark.parametrize("kernel,tol", [("es", 1e-4), ("kb", 1e-4), ("es", 1e-3), ("kb", 1e-5)])
def test_moments_at_narrower_widths(mm, kernel, tol):
    """Dense series (6 events per cell) at looser tolerances: narrower kernels and
    lower polynomial degrees through the moment kernel, against the oracle at tol,
    beside the tap kernel on the same data."""
    N = 1500
    tune = {"spread_direct": 2, "tile": 2048}
    plan = mm.plan_query(N, kernel, tol, "mixed", tune)
    n = int(6 * plan["Mr"])
    w = synth.random_events(2, n, n, seed=int(-np.log10(tol)) * 10 + len(kernel), dp_dtype=torch.float32)
    ref = oracle_coef(w, N)
    for md in (0.0, -1.0):
        c = gpu_coef(mm, w, N, kernel, tol, "mixed", dict(tune, moment_density=md))
        err = series_rel_l2(c, ref)
        assert max(err) <= tol, (kernel, tol, plan["width"], md, err)
