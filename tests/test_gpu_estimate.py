"""GPU checks of mm_estimate (both stages in one call) and its HIP-graph replay.

The one-call form runs the same kernels as mm_nufft1 followed by mm_cov, so its
outputs must equal theirs bit for bit; a few groups are also checked against
the oracle.  Graph replays are checked against an eager call on the same data
every time, with eager work and synchronisation between the replays and new
values written into the same input buffers before each one.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_02842_amd import synth
from tests.helpers import need_gpu, relfro

pytestmark = pytest.mark.gpu

FP64_BAR = 1e-11
MIXED_BAR = 1e-5


@pytest.fixture(scope="module")
def mm():
    need_gpu()
    from paper_2003_02842_amd import mm as m
    return m


def same(a, b):
    """Bitwise equality with NaN == NaN."""
    if a.is_complex():
        return bool(torch.equal(a, b))
    return bool(torch.equal(torch.nan_to_num(a, nan=7.25), torch.nan_to_num(b, nan=7.25)))


def replicates(G, prec):
    w = synth.epps_replicates(G=G, dp_dtype=torch.float32 if prec == "mixed" else torch.float64, device="cuda")
    return w


@pytest.mark.parametrize("basis", ["dirichlet", "fejer"])
@pytest.mark.parametrize("prec,tol", [("mixed", 1e-6), ("fp64", 1e-12)])
def test_estimate_equals_two_calls_and_oracle(mm, basis, prec, tol):
    w = replicates(6, prec)
    Nmax = max(w.Ns)
    c = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, Nmax, "es", tol, prec)
    S1, R1 = mm.cov(c, w.G, w.D, w.Ns, basis)
    coef = torch.empty_like(c)
    S2, R2, _ = mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, w.G, w.D, w.Ns, basis, "es", tol, prec, coef=coef)
    torch.cuda.synchronize()
    assert same(c, coef) and same(S1, S2) and same(R1, R2)
    bar = MIXED_BAR if prec == "mixed" else FP64_BAR
    b = oracle.DIRICHLET if basis == "dirichlet" else oracle.FEJER
    wc = w.to("cpu")
    for g in (0, 5):
        sub = wc.subset(list(range(g * w.D, (g + 1) * w.D)))
        So, Ro = oracle.cov(oracle.coeffs_batch(sub.offsets, sub.t, sub.dp, sub.t0, sub.T, Nmax), 1, w.D, w.Ns, b)
        for q in range(len(w.Ns)):
            assert relfro(S2[q, g].cpu().numpy(), So[q, 0]) <= bar
            assert relfro(R2[q, g].cpu().numpy(), Ro[q, 0]) <= bar


@pytest.mark.parametrize("case", ["replicates-mixed", "replicates-fp64", "wide-mfma", "mfma-sweep", "dense-moments"])
def test_graph_replays_match_eager(mm, case):
    if case == "wide-mfma":
        # D = 60 (1830 pairs) takes the split-BF16 MFMA contraction
        w = synth.random_events(60, 0, 3000, seed=11, T=28_800.0, dp_dtype=torch.float32, device="cuda")
        G, D, Ns, prec, tol = 1, 60, [7, 900], "mixed", 1e-6
    elif case == "mfma-sweep":
        # two groups of 60 and eleven cutoffs: the one-pass sweep on the MFMA path
        w = synth.random_events(120, 0, 3000, seed=13, T=28_800.0, dp_dtype=torch.float32, device="cuda")
        G, D, Ns, prec, tol = 2, 60, [900, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512], "mixed", 1e-6
    elif case == "dense-moments":
        # about 5 events per grid cell: the dense tiles spread from per-cell moments
        w = synth.random_events(40, 20_000, 22_000, seed=17, T=28_800.0, dp_dtype=torch.float32, device="cuda")
        G, D, Ns, prec, tol = 1, 40, [1000], "mixed", 1e-6
    else:
        prec = "mixed" if case.endswith("mixed") else "fp64"
        w = replicates(8, prec)
        G, D, Ns, tol = w.G, w.D, w.Ns, (1e-6 if prec == "mixed" else 1e-12)
    dp0 = w.dp.clone()
    stream = torch.cuda.Stream()
    rdt = torch.float32 if prec == "mixed" else torch.float64
    out = (torch.empty((len(Ns), G, D, D), dtype=rdt, device="cuda"),
           torch.empty((len(Ns), G, D, D), dtype=rdt, device="cuda"))
    ws = torch.empty(mm.estimate_workspace_size(G, D, Ns, "es", tol, prec), dtype=torch.uint8, device="cuda")
    junk = torch.randn(512, 512, device="cuda")
    for rep, scale in enumerate((1.0, 2.0, -0.5, 3.0)):
        w.dp.copy_(dp0 * scale)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, G, D, Ns, "fejer", "es", tol, prec, use_graph=True,
                        out=out, ws=ws)
        stream.synchronize()
        got = (out[0].clone(), out[1].clone())
        # eager work between replays, then the eager result on the same data
        junk = torch.tanh(junk @ junk.T * 1e-3)
        torch.cuda.synchronize()
        S_e, R_e, _ = mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, G, D, Ns, "fejer", "es", tol, prec)
        torch.cuda.synchronize()
        assert same(got[0], S_e) and same(got[1], R_e), (case, rep)
        if rep == 0 and case in ("mfma-sweep", "dense-moments"):
            # the path the case is there for is the one that ran
            mm.profile_reset()
            mm.profile_enable(True)
            mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, G, D, Ns, "fejer", "es", tol, prec)
            torch.cuda.synchronize()
            mm.profile_enable(False)
            assert mm.profile_read("k_sweep_reduce" if case == "mfma-sweep" else "k_spread_mom")[1] >= 1
    # the default stream path (side stream inside the binding) replays the same way
    S_d, R_d, _ = mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, G, D, Ns, "fejer", "es", tol, prec, use_graph=True,
                              out=out, ws=ws)
    torch.cuda.synchronize()
    assert same(S_d, S_e) and same(R_d, R_e)
    mm.graph_cache_clear()


def test_graph_with_coefficient_output_and_new_cutoffs(mm):
    w = replicates(4, "mixed")
    Nmax = max(w.Ns)
    coef = torch.empty((w.S, Nmax + 1), dtype=torch.complex64, device="cuda")
    stream = torch.cuda.Stream()
    results = []
    for Ns in (w.Ns, w.Ns[-5:], w.Ns):
        with torch.cuda.stream(stream):
            S, R, _ = mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, w.G, w.D, Ns, "dirichlet", "es", 1e-6, "mixed",
                                  use_graph=True, coef=coef)
        stream.synchronize()
        c_ref = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, max(Ns), "es", 1e-6, "mixed")
        S_ref, R_ref = mm.cov(c_ref, w.G, w.D, Ns, "dirichlet")
        torch.cuda.synchronize()
        assert same(coef[:, :max(Ns) + 1], c_ref) and same(S, S_ref) and same(R, R_ref)
        results.append(S)
    assert same(results[0], results[2])
    mm.graph_cache_clear()


@pytest.mark.parametrize("basis", ["dirichlet", "fejer"])
@pytest.mark.parametrize("D,N,tune", [(300, 3000, None), (1100, 3000, None), (769, 3000, None), (300, 100, None),
                                      (45, 700, None), (1100, 3000, {"sigma": 1.55, "tile": 2048})])
def test_fused_split_agrees_with_two_calls(mm, basis, D, N, tune):
    """With no coefficient output, one group and one cutoff on the MFMA path, the
    FFT's row pass writes the contraction's BF16 operands itself, row k1 of the FFT
    matrix as one run of columns (coefficient k1 + L1 k2 at column k1 K2 + k2).
    The contraction then sums the same products in another column order, so Sigma
    and R must agree with the two-call form's to FP32 summation rounding (4e-6,
    four times the mixed contraction's error against FP64 at D = 2000) rather than
    bit for bit (128- and 256-wide SYRK tiles, the smallest D of the MFMA path and
    of the 256-wide kernel, a short k range, ragged last tile rows, empty series,
    the tuned plan);
    graph replays must equal the eager call bit for bit; and the oracle on a few
    series."""
    w = synth.random_events(D, 0, 1500, seed=4040 + D + N, dp_dtype=torch.float32, device="cuda")
    c = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, N, "es", 1e-6, "mixed", tune)
    S1, R1 = mm.cov(c, 1, D, [N], basis)
    S2, R2, ws = mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, 1, D, [N], basis, "es", 1e-6, "mixed", tune)
    torch.cuda.synchronize()
    assert relfro(S2.cpu().numpy(), S1.cpu().numpy()) <= 4e-6
    assert relfro(R2.cpu().numpy(), R1.cpu().numpy()) <= 4e-6
    assert torch.equal(S2, S2.transpose(-1, -2))
    out = (torch.empty_like(S2), torch.empty_like(R2))
    st = torch.cuda.Stream()
    for rep in range(3):
        out[0].fill_(float("nan"))
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, 1, D, [N], basis, "es", 1e-6, "mixed", tune, use_graph=True,
                        ws=ws, out=out)
        st.synchronize()
        assert same(S2, out[0]) and same(R2, out[1]), rep
        torch.cuda.synchronize()
    mm.graph_cache_clear()
    # and against the oracle on four non-empty series (their block of Sigma and R)
    counts = (w.offsets[1:] - w.offsets[:-1]).cpu()
    idx = [i for i in range(D) if counts[i] > 0][:4]
    sub = w.to("cpu").subset(idx)
    b = oracle.DIRICHLET if basis == "dirichlet" else oracle.FEJER
    So, Ro = oracle.cov(oracle.coeffs_batch(sub.offsets, sub.t, sub.dp, sub.t0, sub.T, N), 1, 4, [N], b)
    blk = S2[0, 0][idx][:, idx].cpu().numpy()
    assert relfro(blk, So[0, 0]) <= MIXED_BAR
