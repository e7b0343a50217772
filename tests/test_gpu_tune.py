"""GPU check of the autotuner: the chosen plan comes from the candidate set,
meets the accuracy bar against the oracle, and is served from the cache file on
the second call."""
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


def test_autotune_cross_section(mm, tmp_path):
    from paper_2003_02842_amd import tune
    w = synth.cross_section()
    wd = w.to("cuda")
    N = 5000
    cache = str(tmp_path / "tune.json")
    kw = dict(kernel="es", tol=1e-6, basis="fejer", sigmas=(1.75, 2.0, 2.5), tiles=(1024, 2048), evals=(1, 2),
              reps=2, cache_path=cache)
    best = tune.autotune(wd.offsets, wd.t, wd.dp, w.t0, w.T, N, **kw)
    assert not best["cached"] and best["candidates"] >= 2
    t = best["tuning"]
    assert t["sigma"] in (1.75, 2.0, 2.5) and t["tile"] in (1024, 2048) and t["spread_direct"] in (1, 2)
    again = tune.autotune(wd.offsets, wd.t, wd.dp, w.t0, w.T, N, **kw)
    assert again["cached"] and again["tuning"] == t
    c = mm.nufft1(wd.offsets, wd.t, wd.dp, w.t0, w.T, N, "es", 1e-6, "mixed", t)
    S, R = mm.cov(c, 1, 100, [N], "fejer")
    So, Ro = oracle.cov(oracle.coeffs_batch(w.offsets, w.t, w.dp, w.t0, w.T, N), 1, 100, [N], oracle.FEJER)
    assert relfro(S.cpu().numpy(), So) <= 1e-5
    assert relfro(R.cpu().numpy(), Ro) <= 1e-5


@pytest.mark.parametrize("D,N", [(300, 3000), (1100, 2100)])
def test_autotune_contraction(mm, D, N):
    """The contraction tuner picks a (tile, k-split) from its candidate set; the
    estimate at that shape meets the bar against the oracle (128-wide tiles at
    D = 300, both widths at D = 1100)."""
    from paper_2003_02842_amd import tune
    rng = np.random.default_rng(D)
    k = np.arange(N + 1)
    c = ((rng.normal(size=(D, N + 1)) + 1j * rng.normal(size=(D, N + 1))) / np.sqrt(1 + k / 50.0)).astype(np.complex64)
    c[:, 0] = c[:, 0].real
    cd = torch.from_numpy(c).cuda()
    best = tune.autotune_contraction(cd, D, N, "fejer", splits=(0, 1, 3, 7), reps=2)
    assert best["syrk_tile"] in (128, 256) and best["syrk_splits"] in (0, 1, 3, 7) and best["candidates"] >= 4
    S, R = mm.cov(cd, 1, D, [N], "fejer", tune={"syrk_tile": best["syrk_tile"], "syrk_splits": best["syrk_splits"]})
    So, Ro = oracle.cov(c.astype(np.complex128), 1, D, [N], oracle.FEJER)
    assert relfro(S.cpu().numpy(), So) <= 1e-5
    assert relfro(R.cpu().numpy(), Ro) <= 1e-5
    # every shape, including 256-wide tiles on few stages, gives the oracle's estimate
    for t, sp in ((128, 1), (128, 5), (256, 1), (256, 4)):
        S, _ = mm.cov(cd, 1, D, [N], "fejer", correlation=False, tune={"syrk_tile": t, "syrk_splits": sp})
        assert relfro(S.cpu().numpy(), So) <= 1e-5, (t, sp)
