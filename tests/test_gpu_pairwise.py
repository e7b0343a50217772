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
