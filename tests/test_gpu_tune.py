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
