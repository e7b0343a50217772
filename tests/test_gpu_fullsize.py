"""Parity at the workloads' full sizes, in the launch configuration bench.py times.

Outputs the CPU oracle can compute one by one are sampled (coefficients of a few
series at sampled k; the Sigma/R block of a few series, which depends only on
those series); the rest is checked through properties that hold at any size
(symmetry, positive variances, |R| <= 1, positive semi-definiteness of the Fejer
estimate) and against the FP64 GPU form, itself oracle-checked at smaller sizes.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_02842_amd import synth
from tests.helpers import need_gpu, relfro

pytestmark = pytest.mark.gpu

MIXED_BAR = 1e-5


@pytest.fixture(scope="module")
def mm():
    need_gpu()
    from paper_2003_02842_amd import mm as m
    return m


@pytest.fixture(scope="module")
def universe(mm):
    """The benchmark workload: 2000 assets, ~4.5e8 events, N = 50,000, mixed ES
    tol 1e-6, Fejer basis, the autotuned plan.  Sigma and R come from the call
    bench.py times (mm_estimate with the split fused into the FFT's row pass) and
    must agree with the two-call form's to FP32 summation rounding (the same
    products summed in another column order); the coefficients for sampling come
    from mm_nufft1."""
    from paper_2003_02842_amd.tune import LARGE_UNIVERSE, load_tuned
    w = synth.large_universe(device="cuda")
    N = w.Ns[0]
    tune = load_tuned("large-universe") or dict(LARGE_UNIVERSE)   # the plan bench.py runs
    coef = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, N, "es", 1e-6, "mixed", tune)
    cov2, corr2 = mm.cov(coef, 1, w.S, [N], "fejer", tune=tune)
    cov, corr, ws = mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, 1, w.S, [N], "fejer", "es", 1e-6, "mixed", tune)
    torch.cuda.synchronize()
    assert relfro(cov.cpu().numpy(), cov2.cpu().numpy()) <= 4e-6
    assert relfro(corr.cpu().numpy(), corr2.cpu().numpy()) <= 4e-6
    del cov2, corr2, ws
    return w, N, coef, cov[0, 0].cpu().numpy().astype(np.float64), corr[0, 0].cpu().numpy().astype(np.float64)


def test_universe_sampled_coefficients(universe):
    """Coefficients of the smallest, a median and the densest series (1e4 to
    1e6 events, up to about 6.4 events per grid cell) against the oracle at every
    24th k over 0..N: their relative l2 error (Eq. Der:18 over those k) must be
    within the requested tol = 1e-6."""
    w, N, coef, _, _ = universe
    counts = (w.offsets[1:] - w.offsets[:-1]).cpu()
    order = torch.argsort(counts).tolist()
    picks = [order[0], order[len(order) // 2], order[-1]]
    ks = np.arange(0, N + 1, 24, dtype=np.int64)
    for s in picks:
        tt, dd = w.series(s)
        ref = oracle.coeffs_at(tt.cpu(), dd.cpu(), w.t0, w.T, ks)
        got = coef[s, torch.as_tensor(ks, device=coef.device)].cpu().numpy().astype(np.complex128)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-6, (s, int(counts[s]), err)


def test_universe_sigma_block_vs_oracle(universe):
    """The Sigma/R block of series stratified over the count range -- the
    smallest series and one at each count decile up to about 1e5 events -- against
    the oracle over all k = 0..N (an entry depends only on its pair's series, so
    the block check is exact)."""
    w, N, _, cov, corr = universe
    counts = (w.offsets[1:] - w.offsets[:-1]).cpu()
    order = torch.argsort(counts).tolist()
    idx = [order[0]]
    for q in range(1, 10):
        s = order[(q * len(order)) // 10]
        if counts[s] > 1.2e5:
            break
        idx.append(s)
    assert len(idx) >= 5
    idx = sorted(set(idx))
    sub = w.subset(idx).to("cpu")
    c = oracle.coeffs_batch(sub.offsets, sub.t, sub.dp, sub.t0, sub.T, N)
    So, Ro = oracle.cov(c, 1, len(idx), [N], oracle.FEJER)
    blk = np.ix_(idx, idx)
    assert relfro(cov[blk], So[0, 0]) <= MIXED_BAR
    assert relfro(corr[blk], Ro[0, 0]) <= MIXED_BAR


def test_universe_properties(universe):
    w, N, _, cov, corr = universe
    assert np.array_equal(cov, cov.T)
    assert np.all(np.diag(cov) > 0)
    assert np.all(np.abs(corr) <= 1 + 1e-5)
    np.testing.assert_allclose(np.diag(corr), 1.0, atol=1e-6)
    ev = np.linalg.eigvalsh(cov)
    assert ev.min() >= -1e-5 * ev.max()


def test_universe_vs_fp64_gpu_form(mm, universe):
    w, N, _, cov, corr = universe
    dp64 = w.dp.to(torch.float64)
    c64 = mm.nufft1(w.offsets, w.t, dp64, w.t0, w.T, N, "es", 1e-12, "fp64")
    S64, R64 = mm.cov(c64, 1, w.S, [N], "fejer")
    assert relfro(cov, S64[0, 0].cpu().numpy()) <= MIXED_BAR
    assert relfro(corr, R64[0, 0].cpu().numpy()) <= MIXED_BAR


def test_cross_section_full_size(mm):
    """D = 100 one-factor cross-section over 28,800 s, N = 5000, Fejer, ES, mixed
    (MFMA contraction), all series against the oracle."""
    w = synth.cross_section()
    N = 5000
    wd = w.to("cuda")
    c = mm.nufft1(wd.offsets, wd.t, wd.dp, w.t0, w.T, N, "es", 1e-6, "mixed")
    S, R = mm.cov(c, 1, 100, [N], "fejer")
    ref = oracle.coeffs_batch(w.offsets, w.t, w.dp, w.t0, w.T, N)
    So, Ro = oracle.cov(ref, 1, 100, [N], oracle.FEJER)
    assert relfro(S.cpu().numpy(), So) <= MIXED_BAR
    assert relfro(R.cpu().numpy(), Ro) <= MIXED_BAR


@pytest.mark.parametrize("basis", ["dirichlet", "fejer"])
def test_epps_replicates_full_size_sampled(mm, basis):
    """1000 replicates x 10 assets, 19 cutoffs up to 2000 in one call; eight
    replicates checked against the oracle at every cutoff."""
    w = synth.epps_replicates(device="cuda")
    assert w.G == 1000 and len(w.Ns) == 19
    Nmax = max(w.Ns)
    c = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, Nmax, "es", 1e-6, "mixed")
    S, R = mm.cov(c, w.G, w.D, w.Ns, basis)
    S, R = S.cpu().numpy(), R.cpu().numpy()
    b = oracle.DIRICHLET if basis == "dirichlet" else oracle.FEJER
    for g in (0, 1, 137, 500, 501, 777, 998, 999):
        sub = w.subset(list(range(g * w.D, (g + 1) * w.D))).to("cpu")
        ref = oracle.coeffs_batch(sub.offsets, sub.t, sub.dp, sub.t0, sub.T, Nmax)
        So, Ro = oracle.cov(ref, 1, w.D, w.Ns, b)
        for q in range(len(w.Ns)):
            assert relfro(S[q, g], So[q, 0]) <= MIXED_BAR, (g, w.Ns[q])
            assert relfro(R[q, g], Ro[q, 0]) <= MIXED_BAR, (g, w.Ns[q])
    assert np.all(np.isfinite(S)) and np.all(np.abs(R) <= 1 + 1e-5)
