"""mm_estimate_noalloc (the library's fixed device scratch instead of a workspace
argument) against mm_estimate with a workspace: the same kernels, so Sigma and R
must agree bit for bit; two calls in a row, the second on a smaller input, and a
request beyond the scratch size refused before any launch."""
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


def same(a, b):
    return bool(torch.equal(torch.nan_to_num(a, nan=7.25), torch.nan_to_num(b, nan=7.25)))


def test_noalloc_equals_workspace_form_twice(mm):
    # first call: 300 series at N = 3000, the MFMA contraction (38 MiB of scratch)
    big = synth.random_events(300, 0, 1500, seed=777, dp_dtype=torch.float32, device="cuda")
    args = (big.offsets, big.t, big.dp, big.t0, big.T, 1, 300, [3000], "fejer", "es", 1e-6, "mixed")
    assert mm.estimate_workspace_size(1, 300, [3000], "es", 1e-6, "mixed") <= mm.SCRATCH_BYTES
    S1, R1 = mm.estimate_noalloc(*args)
    Sw, Rw, _ = mm.estimate(*args)
    torch.cuda.synchronize()
    assert same(S1, Sw) and same(R1, Rw)
    # second call, smaller: 6 replicates of 10 series, the 19-cutoff sweep (small-D path)
    w = synth.epps_replicates(G=6, seed=4242, device="cuda")
    args2 = (w.offsets, w.t, w.dp, w.t0, w.T, w.G, w.D, w.Ns, "dirichlet", "es", 1e-6, "mixed")
    out = (torch.full((len(w.Ns), w.G, w.D, w.D), float("nan"), device="cuda"),
           torch.full((len(w.Ns), w.G, w.D, w.D), float("nan"), device="cuda"))
    S2, R2 = mm.estimate_noalloc(*args2, out=out)
    Sw2, Rw2, _ = mm.estimate(*args2)
    torch.cuda.synchronize()
    assert S2.data_ptr() == out[0].data_ptr()
    assert same(S2, Sw2) and same(R2, Rw2)
    # and the oracle on one replicate at every cutoff
    wc = w.to("cpu").subset(list(range(w.D)))
    So, Ro = oracle.cov(oracle.coeffs_batch(wc.offsets, wc.t, wc.dp, wc.t0, wc.T, max(w.Ns)), 1, w.D, w.Ns,
                        oracle.DIRICHLET)
    for q in range(len(w.Ns)):
        assert relfro(S2[q, 0].cpu().numpy(), So[q, 0]) <= 1e-5
        assert relfro(R2[q, 0].cpu().numpy(), Ro[q, 0]) <= 1e-5


def test_noalloc_refuses_beyond_scratch(mm):
    w = synth.random_events(2000, 0, 20, seed=5, dp_dtype=torch.float32, device="cuda")
    assert mm.estimate_workspace_size(1, 2000, [500], "es", 1e-6, "mixed") > mm.SCRATCH_BYTES
    out = (torch.zeros((1, 1, 2000, 2000), device="cuda"), torch.zeros((1, 1, 2000, 2000), device="cuda"))
    with pytest.raises(mm.MMError) as ei:
        mm.estimate_noalloc(w.offsets, w.t, w.dp, w.t0, w.T, 1, 2000, [500], "fejer", "es", 1e-6, "mixed", out=out)
    assert ei.value.status == mm.MM_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert float(out[0].abs().max()) == 0.0   # nothing was launched
