"""GPU checks of mm_matrix_to_csr (the MM algorithm's matrix input form) against
the oracle: offsets, Nyquist cutoffs and the window bit-exact, times exact,
returns to the rounding of one log, and the estimate built on them."""
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


def random_matrices(n, D, seed, hole=0.3):
    rng = np.random.default_rng(seed)
    T = np.sort(rng.uniform(0.0, 28_800.0, size=(n, D)), axis=0)
    P = 100.0 * np.exp(np.cumsum(rng.normal(0, 1e-3, size=(n, D)), axis=0))
    P[rng.random((n, D)) < hole] = np.nan
    T[rng.random((n, D)) < hole / 3] = np.nan
    if D >= 3:
        P[:, 0] = np.nan                        # no observation at all
        T[1:, 1] = np.nan                       # a single observation
    return P, T


def check_against_oracle(mm, P, T, dp_dtype):
    off, t, dp, nyq, info = mm.matrix_to_csr(torch.tensor(P, device="cuda"), torch.tensor(T, device="cuda"),
                                             dp_dtype)
    o_off, o_t, o_dp, o_nyq, o_N, o_win = oracle.matrix_to_csr(P, T)
    assert off.cpu().numpy().tolist() == o_off.tolist()
    assert nyq.cpu().numpy().astype(np.int64).tolist() == o_nyq.tolist()
    assert info["N"] == o_N and (info["t0"], info["T"]) == o_win and info["E"] == o_t.size
    np.testing.assert_array_equal(t.cpu().numpy(), o_t)
    if dp_dtype == torch.float64:
        np.testing.assert_allclose(dp.cpu().numpy(), o_dp, rtol=0, atol=4e-15)
    else:   # one FP64 log difference apart before the rounding to FP32
        np.testing.assert_allclose(dp.cpu().numpy().astype(np.float64), o_dp, rtol=2.0 ** -23, atol=1e-15)
    return off, t, dp, info


@pytest.mark.parametrize("n,D", [(5000, 7), (200, 1500), (1, 3), (3, 1)])
@pytest.mark.parametrize("dp_dtype", [torch.float64, torch.float32])
def test_matrix_to_csr_matches_oracle(mm, n, D, dp_dtype):
    P, T = random_matrices(n, D, seed=n * 7 + D)
    off, t, dp, info = check_against_oracle(mm, P, T, dp_dtype)
    if n == 1:
        assert info["E"] == 0 and info["N"] == oracle.INT32_MAX


@pytest.mark.parametrize("prec,tol,bar", [("mixed", 1e-6, 1e-5), ("fp64", 1e-12, 1e-11)])
def test_matrix_input_estimate_at_nyquist(mm, prec, tol, bar):
    """The whole MM algorithm from its matrix inputs: CSR conversion, Nyquist
    cutoff, both stages; against the oracle on the oracle's own conversion."""
    P, T = random_matrices(3000, 6, seed=5, hole=0.5)
    dt = torch.float32 if prec == "mixed" else torch.float64
    off, t, dp, info = check_against_oracle(mm, P, T, dt)
    N = min(info["N"], 4000)
    S, R, _ = mm.estimate(off, t, dp, info["t0"], info["T"], 1, 6, [N], "fejer", "es", tol, prec)
    o_off, o_t, o_dp, _, _, (t0, t1) = oracle.matrix_to_csr(P, T)
    if prec == "mixed":
        o_dp = o_dp.astype(np.float32).astype(np.float64)
    c = oracle.coeffs_batch(o_off, o_t, o_dp, t0, t1, N)
    So, Ro = oracle.cov(c, 1, 6, [N], oracle.FEJER)
    assert relfro(S.cpu().numpy(), So) <= bar
    assert relfro(R.cpu().numpy(), Ro) <= bar


@pytest.mark.parametrize("case", ["negative-price", "unsorted", "repeated", "all-missing"])
def test_matrix_to_csr_rejects_bad_data(mm, case):
    P, T = random_matrices(50, 4, seed=3, hole=0.0)
    if case == "negative-price":
        P[10, 2] = -1.0
    elif case == "unsorted":
        T[20, 3], T[21, 3] = T[21, 3], T[20, 3] - 1.0
    elif case == "repeated":
        T[30, 2] = T[29, 2]
    else:
        P[:] = np.nan
    with pytest.raises(mm.MMError) as e:
        mm.matrix_to_csr(torch.tensor(P, device="cuda"), torch.tensor(T, device="cuda"))
    assert e.value.status == mm.MM_ERR_DATA
