"""GPU checks of the MFMA contraction alone (mm_cov on given coefficients) against
the oracle's FP64 contraction: the 128-wide tile kernel, the 256-wide kernel with
its split-K count, a ragged last tile row, several cutoffs and both bases."""
import numpy as np
import pytest
import torch

import oracle
from tests.helpers import need_gpu, relfro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mm():
    need_gpu()
    from paper_2003_02842_amd import mm as m
    return m


def random_coefficients(D, N, seed):
    """Seeded complex coefficients with a common factor (so that Sigma has large
    off-diagonal entries) and a decaying spectrum, in the FP32 form the mixed
    path stores."""
    rng = np.random.default_rng(seed)
    k = np.arange(N + 1)
    f = (rng.normal(size=N + 1) + 1j * rng.normal(size=N + 1)) / np.sqrt(1 + k / 50.0)
    load = rng.uniform(0.2, 0.8, size=(D, 1))
    idio = (rng.normal(size=(D, N + 1)) + 1j * rng.normal(size=(D, N + 1))) / np.sqrt(1 + k / 50.0)
    c = load * f[None, :] + 0.5 * idio
    c[:, 0] = c[:, 0].real
    return c.astype(np.complex64)


@pytest.mark.parametrize("D,N,Ns", [(300, 3000, [3000]), (1100, 2100, [700, 2100]), (2100, 1100, [1100])])
@pytest.mark.parametrize("basis,b", [("dirichlet", oracle.DIRICHLET), ("fejer", oracle.FEJER)])
def test_mfma_contraction_matches_oracle(mm, D, N, Ns, basis, b):
    c = random_coefficients(D, N, seed=D + N)
    S, R = mm.cov(torch.from_numpy(c).cuda(), 1, D, Ns, basis)
    So, Ro = oracle.cov(c.astype(np.complex128), 1, D, Ns, b)
    S, R = S.cpu().numpy(), R.cpu().numpy()
    for q in range(len(Ns)):
        assert relfro(S[q, 0], So[q, 0]) <= 1e-5, (D, N, Ns[q], relfro(S[q, 0], So[q, 0]))
        assert relfro(R[q, 0], Ro[q, 0]) <= 1e-5, (D, N, Ns[q], relfro(R[q, 0], Ro[q, 0]))
        assert np.array_equal(S[q, 0], S[q, 0].T)


def test_beyond_32bit_flat_index(mm):
    """D = 46341 (D^2 > 2^31) on the MFMA path with a short k range: the correlation
    step and the split-K reduce index the D x D matrix in 64 bits.  Checked on the
    last row and column (flat indices past 2^31) against an FP64 contraction of the
    same coefficients on the host, and diag(R) = 1."""
    D, N = 46341, 8
    rng = np.random.default_rng(46341)
    c = ((rng.normal(size=(D, N + 1)) + 1j * rng.normal(size=(D, N + 1))) * 0.1).astype(np.complex64)
    c[:, 0] = c[:, 0].real
    S, R = mm.cov(torch.from_numpy(c).cuda(), 1, D, [N], "fejer")
    torch.cuda.synchronize()
    rows = [0, 1, 23170, D - 2, D - 1]
    Sg = S[0, 0][rows].double().cpu().numpy()            # 5 x D
    Rg = R[0, 0][rows].double().cpu().numpy()
    Sc = S[0, 0][:, D - 1].double().cpu().numpy()        # last column
    diagR = torch.diagonal(R[0, 0]).double().cpu().numpy()
    del S, R
    torch.cuda.empty_cache()
    cd = c.astype(np.complex128)
    k = np.arange(N + 1)
    wk = (1.0 - k / N) / (N + 1) * np.where(k == 0, 1.0, 2.0) * (2 * np.pi) ** 2   # Fejer, both signs of k
    ref = (cd[rows] * wk) @ cd.conj().T                    # 5 x D, complex; Sigma is its real part
    ref = ref.real
    var = np.einsum("ik,ik,k->i", cd, cd.conj(), wk).real
    assert relfro(Sg, ref) <= 1e-5
    assert relfro(Sc, ref[-1]) <= 1e-5
    Rref = ref / np.sqrt(var[rows][:, None] * var[None, :])
    assert relfro(Rg, Rref) <= 1e-5
    np.testing.assert_allclose(diagR, 1.0, rtol=0, atol=1e-6)


@pytest.mark.parametrize("D", [1, 5, 23, 44])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_small_d_sweep_matches_oracle(mm, D, prec):
    """The small-D sweep (one workgroup per group, running FP64 sums read off at
    every cutoff) at the sizes that stage the most values per thread (D = 23) and
    the largest D it takes (44), over three groups and five cutoffs, both bases."""
    G, N = 3, 700
    c = np.concatenate([random_coefficients(D, N, seed=D * 10 + g) for g in range(G)])
    if prec == "fp64":
        c = c.astype(np.complex128)
    cd = torch.from_numpy(c).cuda()
    Ns = [1, 17, 300, 301, 700]
    for basis, b in (("dirichlet", oracle.DIRICHLET), ("fejer", oracle.FEJER)):
        S, R = mm.cov(cd, G, D, Ns, basis)
        So, Ro = oracle.cov(c.astype(np.complex128), G, D, Ns, b)
        bar = 1e-5 if prec == "mixed" else 1e-11
        S, R = S.cpu().numpy(), R.cpu().numpy()
        for q in range(len(Ns)):
            for g in range(G):
                assert relfro(S[q, g], So[q, g]) <= bar, (D, Ns[q], g)
                assert relfro(R[q, g], Ro[q, g]) <= bar, (D, Ns[q], g)


@pytest.mark.parametrize("D,N", [(300, 1500), (2100, 600)])
@pytest.mark.parametrize("basis,b", [("dirichlet", oracle.DIRICHLET), ("fejer", oracle.FEJER)])
def test_mfma_sweep_in_one_pass(mm, D, N, basis, b):
    """A sweep of cutoffs on the MFMA path (both tile kernels) in one pass over k:
    segment Gram matrices summed in k order, Sigma read off at each cutoff.  The
    cutoffs come unsorted and with a repeat; every slot against the oracle, and the
    one-pass kernels are the ones that ran."""
    c = random_coefficients(D, N, seed=7 * D + N)
    Ns = [N, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 377, 5, N // 2, N - 1]
    mm.profile_reset()
    mm.profile_enable(True)
    S, R = mm.cov(torch.from_numpy(c).cuda(), 1, D, Ns, basis)
    torch.cuda.synchronize()
    mm.profile_enable(False)
    assert mm.profile_read("k_sweep_reduce")[1] == 1
    So, Ro = oracle.cov(c.astype(np.complex128), 1, D, Ns, b)
    S, R = S.cpu().numpy(), R.cpu().numpy()
    for q in range(len(Ns)):
        assert relfro(S[q, 0], So[q, 0]) <= 1e-5, (D, Ns[q], relfro(S[q, 0], So[q, 0]))
        assert relfro(R[q, 0], Ro[q, 0]) <= 1e-5, (D, Ns[q], relfro(R[q, 0], Ro[q, 0]))
        assert np.array_equal(S[q, 0], S[q, 0].T)
    assert np.array_equal(S[4, 0], S[14, 0])      # the repeated cutoff


def test_mfma_sweep_declined_when_separate_products_cost_less(mm):
    """Two Fejer cutoffs (N/2, N) cost less as two products than as the one-pass
    sweep's two full-width products: the per-cutoff path runs, within the bar."""
    D, N = 300, 1200
    c = random_coefficients(D, N, seed=12)
    mm.profile_reset()
    mm.profile_enable(True)
    S, R = mm.cov(torch.from_numpy(c).cuda(), 1, D, [N // 2, N], "fejer")
    torch.cuda.synchronize()
    mm.profile_enable(False)
    assert mm.profile_read("k_sweep_reduce")[1] == 0
    So, Ro = oracle.cov(c.astype(np.complex128), 1, D, [N // 2, N], oracle.FEJER)
    for q in range(2):
        assert relfro(S[q, 0].cpu().numpy(), So[q, 0]) <= 1e-5


def test_mfma_sweep_groups(mm):
    """The one-pass sweep over two groups of D = 300: each group's slots against
    the oracle (the group offset of the outputs and of the operands)."""
    D, N, G = 300, 900, 2
    c = np.concatenate([random_coefficients(D, N, seed=31), random_coefficients(D, N, seed=32)])
    Ns = [1, 3, 9, 27, 81, 243, 729, 900]
    S, R = mm.cov(torch.from_numpy(c).cuda(), G, D, Ns, "fejer")
    So, Ro = oracle.cov(c.astype(np.complex128), G, D, Ns, oracle.FEJER)
    S, R = S.cpu().numpy(), R.cpu().numpy()
    for q in range(len(Ns)):
        for g in range(G):
            assert relfro(S[q, g], So[q, g]) <= 1e-5, (q, g)
            assert relfro(R[q, g], Ro[q, g]) <= 1e-5, (q, g)
