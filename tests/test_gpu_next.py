"""GPU checks beyond the core path: the zero-padded FFT negative control on the
missing-data and arrival-time representations, and the Epps sweep."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2003_02842_amd import epps, synth
from tests.helpers import need_gpu, relfro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mm():
    need_gpu()
    from paper_2003_02842_amd import mm as m
    return m


def estimate_fp64(mm, w, t, N, basis="dirichlet"):
    S, R, _ = mm.estimate(w.offsets, t, w.dp, w.t0, w.T, w.G, w.D, [N], basis, "es", 1e-12, "fp64")
    return S[0].cpu().numpy(), R[0].cpu().numpy()


def test_snap_times_bit_exact(mm):
    w = synth.bivariate_async()
    span = w.T - w.t0
    for Nstar in (7, 1000, 28_800, 123_457):
        got = mm.snap_times(w.t.cuda(), w.t0, w.T, Nstar).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.snap_times(w.t, w.t0, w.T, Nstar))


def test_zero_padded_fft_matches_on_missing_data(mm):
    """Missing-data representation: every time is already one of the n grid
    points, so moving times to the grid changes nothing and the zero-padded FFT
    agrees with the NUFFT and the oracle."""
    w = synth.missing_data().to("cuda")
    n = 10_000
    N = w.Ns[0] // 2
    snapped = mm.snap_times(w.t, w.t0, w.T, n)
    assert float((snapped - w.t).abs().max()) < 1e-12 * w.T
    S_n, R_n = estimate_fp64(mm, w, w.t, N)
    S_z, R_z = estimate_fp64(mm, w, snapped, N)
    wc = w.to("cpu")
    So, Ro = oracle.cov(oracle.coeffs_batch(wc.offsets, wc.t, wc.dp, wc.t0, wc.T, N), 1, 2, [N], oracle.DIRICHLET)
    assert relfro(S_n, So[0]) <= 1e-11 and relfro(R_n, Ro[0]) <= 1e-11
    assert relfro(S_z, So[0]) <= 1e-10 and relfro(R_z, Ro[0]) <= 1e-10


def test_zero_padded_fft_fails_under_arrival_times(mm):
    """Arrival-time representation (Poisson sampling at 1/15 and 1/30 per second):
    a zero-padded FFT grid of 2N+1 points (the modes up to N) moves the events by
    up to half a grid step and misses the oracle by percents, while the NUFFT
    agrees to 1e-11."""
    w = synth.bivariate_async().to("cuda")
    wc = w.to("cpu")
    N = 200
    S_n, R_n = estimate_fp64(mm, w, w.t, N)
    S_z, R_z = estimate_fp64(mm, w, mm.snap_times(w.t, w.t0, w.T, 2 * N + 1), N)
    So, Ro = oracle.cov(oracle.coeffs_batch(wc.offsets, wc.t, wc.dp, wc.t0, wc.T, N), 1, 2, [N], oracle.DIRICHLET)
    assert relfro(S_n, So[0]) <= 1e-11 and relfro(R_n, Ro[0]) <= 1e-11
    assert relfro(S_z, So[0]) > 1e-3, relfro(S_z, So[0])


def test_epps_sweep_follows_the_poisson_model(mm):
    """100 replicates of a bivariate GBM (rho = 0.35) under Poisson sampling at
    lam = 1/5 per second: the mean Dirichlet correlation over sampling intervals
    1..100 s fits Eq. Der:21 with c near rho (lam fixed), and the Fejer curve lies
    above the Dirichlet one at the shortest interval (loose shape check)."""
    rho, lam = 0.35, 1 / 5
    w = synth.epps_pairs(G=100, rho=rho, lam=lam, device="cuda")
    dts = [1, 2, 3, 5, 8, 13, 21, 34, 55, 100]
    Ns, R_d = epps.sweep(w.offsets, w.t, w.dp, w.t0, w.T, w.G, 2, dts, "dirichlet")
    _, R_f = epps.sweep(w.offsets, w.t, w.dp, w.t0, w.T, w.G, 2, dts, "fejer")
    r_d = R_d[:, :, 0, 1].double().mean(1).cpu().numpy()
    r_f = R_f[:, :, 0, 1].double().mean(1).cpu().numpy()
    dt_of_N = np.array([epps.interval_for_cutoff(w.T - w.t0, N) for N in Ns])
    c, _, _ = epps.fit_epps(dt_of_N, r_d, lam=lam)
    assert abs(c - rho) < 0.05, (c, r_d)
    assert r_f[-1] > r_d[-1]                                # largest N = shortest interval
    assert np.all(np.diff(r_d[::-1]) >= -0.02)               # correlation grows with the interval
