"""Host-side checks of the C ABI: the library loads without a GPU, exports every
entry point declared in include/mm.h, rejects invalid arguments before any device
work, and plans grids and widths per the paper's rules."""
import ctypes
import json
import os
import re

import pytest
import torch  # noqa: F401  (load torch's HIP runtime first)

from paper_2003_02842_amd import mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mm.lib()
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(mm.EXPORTED)


def test_contraction_tuning_changes_only_the_workspace_shape():
    """The tile and k-split choices size the split-K partials; 0 keeps the model's."""
    auto = mm.cov_workspace_size(1, 2000, 50_000, 1, "mixed")
    assert mm.cov_workspace_size(1, 2000, 50_000, 1, "mixed", {"syrk_tile": 0, "syrk_splits": 0}) == auto
    one = mm.cov_workspace_size(1, 2000, 50_000, 1, "mixed", {"syrk_tile": 256, "syrk_splits": 1})
    eight = mm.cov_workspace_size(1, 2000, 50_000, 1, "mixed", {"syrk_tile": 256, "syrk_splits": 8})
    assert one < eight and eight - one == 7 * 36 * 256 * 256 * 4     # 36 lower tiles of 256 x 256 FP32
    small = mm.cov_workspace_size(1, 2000, 50_000, 1, "mixed", {"syrk_tile": 128, "syrk_splits": 1})
    assert small != one


def test_status_strings():
    for s in range(7):
        assert mm.lib().mm_status_string(s)


def _nufft_raw(**kw):
    a = dict(S=2, offsets=1, t=1, dp=1, dpf=0, t0=0.0, T=1.0, N=10, kernel=2, tol=1e-6, prec=1, tune=None, coef=1,
             ldc=11, ws=256, wsb=1 << 40, validate=0, stream=None)
    a.update(kw)
    P = ctypes.c_void_p
    return mm.lib().mm_nufft1(a["S"], P(a["offsets"]), P(a["t"]), P(a["dp"]), a["dpf"], a["t0"], a["T"], a["N"],
                              a["kernel"], a["tol"], a["prec"], a["tune"], P(a["coef"]), a["ldc"], P(a["ws"]),
                              a["wsb"], a["validate"], a["stream"])


@pytest.mark.parametrize("kw,status", [
    (dict(S=-1), mm.MM_ERR_ARG), (dict(N=0), mm.MM_ERR_ARG), (dict(T=0.0), mm.MM_ERR_ARG),
    (dict(T=float("nan")), mm.MM_ERR_ARG), (dict(ldc=10), mm.MM_ERR_ARG), (dict(offsets=0), mm.MM_ERR_ARG),
    (dict(coef=0), mm.MM_ERR_ARG), (dict(dpf=2), mm.MM_ERR_ARG), (dict(kernel=7), mm.MM_ERR_ARG),
    (dict(prec=3), mm.MM_ERR_ARG), (dict(tol=1e-7), mm.MM_ERR_TOL), (dict(tol=0.5), mm.MM_ERR_TOL),
    (dict(prec=0, tol=1e-15), mm.MM_ERR_TOL), (dict(tol=float("nan")), mm.MM_ERR_TOL),
    (dict(wsb=16), mm.MM_ERR_WORKSPACE), (dict(ws=0), mm.MM_ERR_WORKSPACE), (dict(ws=257), mm.MM_ERR_ARG),
    (dict(S=0), mm.MM_OK),
])
def test_nufft1_rejects_before_launch(kw, status):
    assert _nufft_raw(**kw) == status


def _cov_raw(**kw):
    a = dict(G=1, D=3, coef=1, ldc=11, Ns=[5], basis=0, prec=1, tune=None, cov=1, corr=0, ws=0, wsb=0)
    a.update(kw)
    P = ctypes.c_void_p
    arr = (ctypes.c_int32 * max(1, len(a["Ns"])))(*a["Ns"]) if a["Ns"] is not None else None
    n = a.get("nN", len(a["Ns"]) if a["Ns"] is not None else 1)
    tune = ctypes.byref(mm._tuning(a["tune"])) if a["tune"] is not None else None
    return mm.lib().mm_cov(a["G"], a["D"], P(a["coef"]), a["ldc"], arr, n, a["basis"], a["prec"], tune,
                           P(a["cov"]), P(a["corr"]), P(a["ws"]), a["wsb"], None)


@pytest.mark.parametrize("kw,status", [
    (dict(G=0), mm.MM_ERR_ARG), (dict(D=0), mm.MM_ERR_ARG), (dict(coef=0), mm.MM_ERR_ARG),
    (dict(cov=0), mm.MM_ERR_ARG), (dict(Ns=[11]), mm.MM_ERR_ARG), (dict(Ns=[0]), mm.MM_ERR_ARG),
    (dict(Ns=None), mm.MM_ERR_ARG), (dict(nN=0), mm.MM_ERR_ARG), (dict(nN=129, Ns=[1] * 129), mm.MM_ERR_ARG),
    (dict(basis=2), mm.MM_ERR_ARG), (dict(prec=9), mm.MM_ERR_ARG),
    (dict(D=200, ldc=5001, Ns=[5000]), mm.MM_ERR_WORKSPACE),
    (dict(tune={"syrk_tile": 64}), mm.MM_ERR_ARG), (dict(tune={"syrk_splits": -1}), mm.MM_ERR_ARG),
    (dict(D=200, ldc=5001, Ns=[5000], tune={"syrk_tile": 128, "syrk_splits": 3}), mm.MM_ERR_WORKSPACE),
])
def test_cov_rejects_before_launch(kw, status):
    assert _cov_raw(**kw) == status


def test_min_halfwidths_printed_in_paper():
    g = GOLDEN["min_spread_halfwidth"]
    for key, kern in (("gaussian", "g"), ("kaiser_bessel", "kb"), ("es", "es")):
        info = mm.plan_query(100, kern, g[key]["tol"], "fp64")
        assert info["msp"] == g[key]["msp"], key


def test_grid_length_rule():
    """M_r = sigma (2N+1) (Sec. 2.2.5); ours is the smallest even 2,3,5-smooth
    length not below it, so it equals the printed value when that is smooth."""
    for c in GOLDEN["grid_length_examples"]["cases"]:
        Mr = mm.plan_query(c["N"], "es", 1e-6, "fp64")["Mr"]
        assert Mr >= c["Mr"]
        n, smooth = c["Mr"], True
        for p in (2, 3, 5):
            while n % p == 0:
                n //= p
        smooth = (n == 1)
        if smooth:
            assert Mr == c["Mr"]
        assert Mr % 2 == 0


@pytest.mark.parametrize("N", [1, 2, 3, 7, 100, 5000, 50000, 123457])
@pytest.mark.parametrize("kern,tol,prec", [("es", 1e-12, "fp64"), ("g", 1e-6, "mixed"), ("kb", 1e-9, "fp64"),
                                           ("es", 1e-1, "mixed")])
def test_plan_invariants(N, kern, tol, prec):
    p = mm.plan_query(N, kern, tol, prec)
    assert p["Mr"] >= 2 * (2 * N + 1) and p["Mr"] >= 2 * p["width"] and p["Mr"] % 2 == 0
    assert p["L1"] * p["L2"] * 2 == p["Mr"] and p["L1"] <= p["L2"] <= 2048
    for n in (p["L1"], p["L2"]):
        for q in (2, 3, 5):
            while n % q == 0:
                n //= q
        assert n == 1


def test_width_grows_as_tolerance_tightens():
    for kern in ("g", "kb", "es"):
        ws = [mm.plan_query(1000, kern, tol, "fp64")["width"] for tol in (1e-1, 1e-3, 1e-6, 1e-9, 1e-12, 1e-14)]
        assert ws == sorted(ws) and ws[0] < ws[-1]


@pytest.mark.parametrize("kern", ["es", "kb", "g"])
@pytest.mark.parametrize("tol", [1e-1, 1e-2, 1e-4, 1e-6])
def test_mixed_default_width_meets_estimate(kern, tol):
    """On the mixed path the planner takes the smallest width whose a-priori
    error estimate is within tol; one tap less would not be."""
    p = mm.plan_query(20_000, kern, tol, "mixed")
    assert p["est_err"] <= tol
    step = 1 if kern == "es" else 2
    if p["width"] - step >= (3 if kern == "kb" else 2):
        q = mm.plan_query(20_000, kern, tol, "mixed", {"width": p["width"] - step})
        assert q["est_err"] > tol


@pytest.mark.parametrize("kern", ["es", "kb", "g"])
def test_error_estimate_decreases_with_width(kern):
    """The aliasing/truncation estimate (the FP64 path's) falls with every added
    tap.  The mixed path's estimate also covers FP32 rounding, which the
    deconvolution amplifies more as the kernel widens: it is never below the
    FP64 one, stops falling, and never drops under one unit of 2^-24."""
    step = 1 if kern == "es" else 2
    w0 = 3 if kern == "kb" else 2
    ws = range(w0, 17, step)
    ests = [mm.plan_query(500, kern, 1e-6, "fp64", {"width": w})["est_err"] for w in ws]
    assert all(b < a for a, b in zip(ests, ests[1:]))
    mixed = [mm.plan_query(500, kern, 1e-6, "mixed", {"width": w})["est_err"] for w in ws]
    assert all(m >= f for m, f in zip(mixed, ests))
    assert mixed[0] == ests[0] and min(mixed) >= 2.0 ** -24
    assert mixed[-1] > ests[-1]


def test_rounding_floor_refuses_low_oversampling():
    """At sigma = 1.25 the deconvolution amplifies FP32 rounding by ~40 (rms over
    the band), so no width meets tol 1e-6 on the mixed path, and FP64 cannot
    reach 1e-12 there; at sigma = 1.55 the mixed plan exists and its estimate
    covers the rounding term 2^-24 * 2 * rms amplification (about 3.5e-7)."""
    for kern in ("es", "kb"):
        with pytest.raises(mm.MMError, match="status 3"):
            mm.plan_query(2700, kern, 1e-6, "mixed", {"sigma": 1.25})
        with pytest.raises(mm.MMError, match="status 3"):
            mm.plan_query(2700, kern, 1e-12, "fp64", {"sigma": 1.25})
    p = mm.plan_query(50_000, "es", 1e-6, "mixed", {"sigma": 1.55})
    assert p["width"] == 9 and 3e-7 < p["est_err"] <= 1e-6
    # explicit widths bypass the search, and the estimate then reports the floor
    q = mm.plan_query(2700, "es", 1e-6, "mixed", {"sigma": 1.25, "width": 12})
    assert q["est_err"] > 2e-6


def test_fp64_default_is_paper_rule():
    for kern, tol in (("es", 1e-12), ("kb", 1e-9), ("g", 1e-6)):
        a = mm.plan_query(1000, kern, tol, "fp64")
        b = mm.plan_query(1000, kern, tol, "mixed" if tol >= 1e-6 else "fp64", {"width": -1})
        assert a["width"] == b["width"]


def _est_raw(**kw):
    a = dict(G=2, D=3, offsets=1, t=1, dp=1, dpf=0, t0=0.0, T=1.0, Ns=[5, 9], basis=1, kernel=2, tol=1e-6, prec=1,
             tune=None, coef=0, ldc=0, cov=1, corr=0, ws=256, wsb=1 << 40, graph=0, stream=None)
    a.update(kw)
    P = ctypes.c_void_p
    arr = (ctypes.c_int32 * max(1, len(a["Ns"])))(*a["Ns"]) if a["Ns"] is not None else None
    n = a.get("nN", len(a["Ns"]) if a["Ns"] is not None else 1)
    return mm.lib().mm_estimate(a["G"], a["D"], P(a["offsets"]), P(a["t"]), P(a["dp"]), a["dpf"], a["t0"], a["T"],
                                arr, n, a["basis"], a["kernel"], a["tol"], a["prec"], a["tune"], P(a["coef"]),
                                a["ldc"], P(a["cov"]), P(a["corr"]), P(a["ws"]), a["wsb"], a["graph"],
                                P(a["stream"]) if a["stream"] else None)


@pytest.mark.parametrize("kw,status", [
    (dict(G=0), mm.MM_ERR_ARG), (dict(D=0), mm.MM_ERR_ARG), (dict(t=0), mm.MM_ERR_ARG), (dict(cov=0), mm.MM_ERR_ARG),
    (dict(Ns=None), mm.MM_ERR_ARG), (dict(Ns=[0]), mm.MM_ERR_ARG), (dict(nN=0), mm.MM_ERR_ARG),
    (dict(basis=5), mm.MM_ERR_ARG), (dict(dpf=3), mm.MM_ERR_ARG), (dict(graph=2), mm.MM_ERR_ARG),
    (dict(graph=1), mm.MM_ERR_ARG),                      # graphs need a non-default stream
    (dict(T=-1.0), mm.MM_ERR_ARG), (dict(coef=1, ldc=5), mm.MM_ERR_ARG), (dict(tol=1e-9), mm.MM_ERR_TOL),
    (dict(G=300, D=300), mm.MM_ERR_UNSUPPORTED), (dict(wsb=1024), mm.MM_ERR_WORKSPACE), (dict(ws=0), mm.MM_ERR_WORKSPACE),
    (dict(ws=300), mm.MM_ERR_ARG),
])
def test_estimate_rejects_before_launch(kw, status):
    assert _est_raw(**kw) == status


def test_estimate_workspace_covers_both_stages():
    G, D, Ns = 4, 10, [1, 7, 2000]
    est = mm.estimate_workspace_size(G, D, Ns, "es", 1e-6, "mixed")
    nufft = mm.nufft1_workspace_size(G * D, max(Ns), "es", 1e-6, "mixed")
    coef = G * D * (max(Ns) + 1) * 8
    assert est >= nufft + coef + mm.cov_workspace_size(G, D, max(Ns), len(Ns), "mixed")


def test_planner_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The planner (mm_plan.cpp) built for the host with ASan and UBSan plans ~19k
    combinations of cutoff, kernel, tolerance, precision and tuning, valid and not,
    and checks what every accepted plan promises (tests/plan_sanitize.cpp)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    csrc = os.path.join(ROOT, "paper_2003_02842_amd", "csrc")
    exe = str(tmp_path / "plan_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           "-I", csrc, os.path.join(csrc, "mm_plan.cpp"), os.path.join(ROOT, "tests", "plan_sanitize.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "0 failed checks" in r.stdout and "ERROR" not in r.stderr and "runtime error" not in r.stderr
