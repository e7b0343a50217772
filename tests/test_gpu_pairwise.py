"""GPU parity of mm_cov_pairwise (per-asset cutoffs, N_ij = min(N_i, N_j))."""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_02842_amd import synth
from tests.helpers import need_gpu, relfro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mm():
    need_gpu()
    from paper_2003_02842_amd import mm as m
    return m


@pytest.mark.parametrize("basis", ["dirichlet", "fejer"])
@pytest.mark.parametrize("D,distinct,prec,tol,bar", [(6, 6, "fp64", 1e-12, 1e-11), (6, 6, "mixed", 1e-6, 1e-5),
                                                     (50, 4, "mixed", 1e-6, 1e-5)])
def test_pairwise_matches_oracle(mm, basis, D, distinct, prec, tol, bar):
    w = synth.random_events(2 * D, 100, 1500, seed=D + distinct,
                            dp_dtype=torch.float64 if prec == "fp64" else torch.float32)
    rng = np.random.default_rng(D)
    levels = rng.integers(30, 900, size=distinct)
    Ni = [int(levels[i % distinct]) for i in range(D)]
    G = 2
    wd = w.to("cuda")
    Nmax = max(Ni)
    c = mm.nufft1(wd.offsets, wd.t, wd.dp, w.t0, w.T, Nmax, "es", tol, prec)
    S, R = mm.cov_pairwise(c, G, D, Ni, basis)
    ref = oracle.coeffs_batch(w.offsets, w.t, w.dp, w.t0, w.T, Nmax)
    b = oracle.DIRICHLET if basis == "dirichlet" else oracle.FEJER
    So, Ro = oracle.cov_pairwise(ref, G, D, Ni, b)
    assert relfro(S.cpu().numpy(), So) <= bar
    assert relfro(R.cpu().numpy(), Ro) <= bar
    assert np.array_equal(S.cpu().numpy(), S.cpu().numpy().transpose(0, 2, 1))


def _block_vs_oracle(S, R, ref, G, idx, Ni, b, bar):
    """The pairwise block of the assets idx depends only on their coefficients and
    cutoffs, so the oracle computes it exactly from them."""
    for g in range(G):
        rows = [g * len(Ni) + i for i in idx]
        So, Ro = oracle.cov_pairwise(ref[rows], 1, len(idx), [Ni[i] for i in idx], b)
        blk = np.ix_(idx, idx)
        assert relfro(S[g][blk], So[0]) <= bar, (g, relfro(S[g][blk], So[0]))
        assert relfro(R[g][blk], Ro[0]) <= bar, (g, relfro(R[g][blk], Ro[0]))


@pytest.mark.parametrize("basis", ["dirichlet", "fejer"])
@pytest.mark.parametrize("prec,tol,bar", [("mixed", 1e-6, 1e-5), ("fp64", 1e-12, 1e-11)])
def test_pairwise_one_cutoff_per_asset(mm, basis, prec, tol, bar):
    """D = 300 with 300 distinct cutoffs (the one-pass product over assets sorted by
    cutoff; on the mixed path the 128-wide MFMA tiles), two groups, in no particular
    order; a 14-asset block spanning the cutoff range against the oracle."""
    D, G = 300, 2
    w = synth.random_events(G * D, 50, 1200, seed=300 + len(prec),
                            dp_dtype=torch.float64 if prec == "fp64" else torch.float32)
    rng = np.random.default_rng(77)
    Ni = [int(v) for v in rng.permutation(np.arange(40, 40 + 3 * D, 3))]
    Nmax = max(Ni)
    wd = w.to("cuda")
    c = mm.nufft1(wd.offsets, wd.t, wd.dp, w.t0, w.T, Nmax, "es", tol, prec)
    S, R = mm.cov_pairwise(c, G, D, Ni, basis)
    S, R = S.cpu().numpy(), R.cpu().numpy()
    assert np.array_equal(S, S.transpose(0, 2, 1))
    order = np.argsort(Ni)
    idx = sorted(set(int(order[q]) for q in np.linspace(0, D - 1, 14).astype(int)))
    ref = oracle.coeffs_batch(w.offsets, w.t, w.dp, w.t0, w.T, Nmax)
    b = oracle.DIRICHLET if basis == "dirichlet" else oracle.FEJER
    _block_vs_oracle(S, R, ref, G, idx, Ni, b, bar)


def test_pairwise_large_universe_every_cutoff_distinct(mm):
    """The large universe (2000 assets, N up to 50,000) with its own cutoff for
    every asset, log-spaced over [1000, 50000] and shuffled: the mixed one-pass
    product (256-wide MFMA tiles) against the FP64 one-pass form over the whole
    matrix, and an eight-asset block of the smallest series against the oracle."""
    from paper_2003_02842_amd.tune import LARGE_UNIVERSE
    w = synth.large_universe(device="cuda")
    D, N = w.S, 50_000
    rng = np.random.default_rng(2000)
    Ni = [int(v) for v in rng.permutation(np.unique(np.round(np.geomspace(1000, N, 2600)).astype(int))[:D])]
    assert len(set(Ni)) == D and max(Ni) <= N
    c = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, N, "es", 1e-6, "mixed", dict(LARGE_UNIVERSE))
    S, R = mm.cov_pairwise(c, 1, D, Ni, "fejer")
    torch.cuda.synchronize()
    del c
    c64 = mm.nufft1(w.offsets, w.t, w.dp.double(), w.t0, w.T, N, "es", 1e-12, "fp64")
    S64, R64 = mm.cov_pairwise(c64, 1, D, Ni, "fejer")
    torch.cuda.synchronize()
    del c64
    S, R, S64, R64 = (x.cpu().numpy().astype(np.float64) for x in (S, R, S64, R64))
    assert np.array_equal(S, S.transpose(0, 2, 1))
    assert relfro(S, S64) <= 1e-5 and relfro(R, R64) <= 1e-5
    counts = (w.offsets[1:] - w.offsets[:-1]).cpu()
    idx = sorted(torch.argsort(counts)[:8].tolist())
    sub = w.subset(idx).to("cpu")
    refN = max(Ni[i] for i in idx)
    ref = oracle.coeffs_batch(sub.offsets, sub.t, sub.dp, sub.t0, sub.T, refN)
    So, Ro = oracle.cov_pairwise(ref, 1, len(idx), [Ni[i] for i in idx], oracle.FEJER)
    blk = np.ix_(idx, idx)
    assert relfro(S[0][blk], So[0]) <= 1e-5 and relfro(R[0][blk], Ro[0]) <= 1e-5
