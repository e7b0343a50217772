#!/usr/bin/env python3
"""Throughput of the Malliavin-Mancino hot path on one MI355X.

One step = the whole path over one batch of synthetic input already resident in
HBM: the type-1 NUFFT of every series (spreading, two-pass grid FFT,
deconvolution) and the Fejer contraction with correlation, in the mixed form
(FP32 NUFFT, split-BF16 MFMA contraction), as one mm_estimate call with no
coefficient output (the FFT's row pass writes the contraction's operands).

Workload (default): the large-universe case -- D = 2000 assets of a 3-factor
GBM, event counts log-uniform in [1e4, 1e6] (about 4.3e8 events), horizon
28,800 s, N = 50,000, exponential-of-semicircle kernel.

Printed: one JSON line (rank 0).  `value` is events/s of the mixed form;
alongside: contraction TFLOP/s (GEMM-equivalent 2 D^2 (2N+1) flops), the
speed-up over the plain FP64 GPU form (one launch chain per series, FP64
contraction) on the same input, the relative Frobenius error of Sigma and R
against the FP64 GPU form at tol 1e-12, the roofline of the dominant kernel
from HIP events recorded around every launch in a profiled pass after the timed
region (the timed region itself runs uninstrumented), the CPU oracle timed on a
bounded, count-stratified sample of the same workload, and the cross-section and
Monte Carlo replicates workloads through mm_estimate (graph replay and eager).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
SPREAD_PAIR = "k_spread_poly+k_spread_mom"
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--D", type=int, default=2000)
    ap.add_argument("--n-lo", type=float, default=1e4)
    ap.add_argument("--n-hi", type=float, default=1e6)
    ap.add_argument("--N", type=int, default=50_000)
    ap.add_argument("--kernel", default="es")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--basis", default="fejer")
    ap.add_argument("--seed", type=int, default=20200310)
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain FP64 GPU form (and, for the other workloads, the per-cutoff re-run)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU-oracle sample time (three runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="leave the cross-section and replicates results out of the default line")
    ap.add_argument("--width", type=int, default=0, help="override the spreading width")
    ap.add_argument("--sigma", type=float, default=0.0, help="override the oversampling factor")
    ap.add_argument("--untuned", action="store_true",
                    help="the planner's defaults (sigma = 2) instead of the autotuned large-universe plan")
    ap.add_argument("--workload", default="large-universe", choices=("large-universe", "replicates", "cross-section", "pairwise"),
                    help="large-universe (the default bench line), or the Monte Carlo replicates / 100-asset "
                         "cross-section timed through mm_estimate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (scales FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--summarize", nargs="+", metavar=("KIND", "DIR"),
                    help="print the Markdown table of rocprofv3 CSV output instead of benchmarking: "
                         "'trace DIR' (kernel durations), 'traffic FETCH_DIR WRITE_DIR COPYF_DIR COPYW_DIR' "
                         "(HBM bytes per launch, scaled by the copy's counters), 'counters DIR' (per-dispatch "
                         "medians of every counter)")
    return ap.parse_args()


def _short_kernel(name: str) -> str:
    """mm::k_spread_poly<float, 9, 4>(...) -> k_spread_poly"""
    n = name.split("(")[0].split("<")[0].split("::")[-1].split()
    return n[-1] if n else name.strip()


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def _median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def _counter_medians(d):
    """{kernel: {counter: median over dispatches of the per-dispatch sum}} of a counter_collection CSV."""
    import csv
    per = {}
    for f in _csvs(d, "counter_collection.csv"):
        for row in csv.DictReader(open(f)):
            k = _short_kernel(row.get("Kernel_Name", ""))
            key = (row.get("Counter_Name"), row.get("Dispatch_Id"))
            per.setdefault(k, {}).setdefault(key, 0.0)
            per[k][key] += float(row.get("Counter_Value", 0) or 0)
    out = {}
    for k, d2 in per.items():
        byc = {}
        for (c, _), v in d2.items():
            byc.setdefault(c, []).append(v)
        out[k] = {c: (_median(v), len(v)) for c, v in byc.items()}
    return out


def summarize(args):
    """Markdown tables from rocprofv3 CSV output (the files under profiles/ are made with this)."""
    import csv
    kind, dirs = args[0], args[1:]
    if kind == "trace":
        durs = {}
        for f in _csvs(dirs[0], "kernel_trace.csv"):
            for row in csv.DictReader(open(f)):
                k = _short_kernel(row.get("Kernel_Name", ""))
                if not k.startswith("k_"):
                    continue
                durs.setdefault(k, []).append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
        print("| kernel | calls | avg | median | min | max | total |")
        print("|---|---|---|---|---|---|---|")
        for k, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
            print("| %s | %d | %.1f | %.1f | %.1f | %.1f | %.1f |" % (k, len(v), sum(v) / len(v), _median(v), min(v),
                                                                      max(v), sum(v)))
    elif kind == "traffic":
        fetch, write, copyf, copyw = (_counter_medians(d) for d in dirs[:4])

        def copy_kib(m, c):
            vals = [v[c][0] for v in m.values() if c in v]
            return max(vals) if vals else None
        cf, cw = copy_kib(copyf, "FETCH_SIZE"), copy_kib(copyw, "WRITE_SIZE")
        fr, wr = (1 << 20) / cf, (1 << 20) / cw      # bytes a 1 GiB copy moves, per KiB counted
        print("Calibration: a 1 GiB device-to-device copy reads FETCH_SIZE = %d KiB and WRITE_SIZE = %d KiB, so "
              "bytes = FETCH_SIZE x 1024 x %.3f and WRITE_SIZE x 1024 x %.3f." % (cf, cw, fr, wr))
        print()
        print("source_sha256_16: %s" % source_hash(_tuned_large_universe()))
        print()
        print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB | traffic_bytes |")
        print("|---|---|---|---|---|---|---|")
        for k in sorted(set(fetch) | set(write)):
            if not k.startswith("k_"):
                continue
            f, n = fetch.get(k, {}).get("FETCH_SIZE", (0.0, 0))
            w, _ = write.get(k, {}).get("WRITE_SIZE", (0.0, 0))
            rb, wb = f * 1024 * fr, w * 1024 * wr
            print("| %s | %d | %.0f | %.0f | %.1f | %.1f | %.0f |" % (k, n, f, w, rb / 1e6, wb / 1e6, rb + wb))
    elif kind == "counters":
        m = _counter_medians(dirs[0])
        cs = sorted({c for v in m.values() for c in v})
        print("| kernel | " + " | ".join(cs) + " |")
        print("|---|" + "---|" * len(cs))
        for k in sorted(m):
            if k.startswith("k_"):
                print("| %s | " % k + " | ".join("%.4g" % m[k][c][0] if c in m[k] else "" for c in cs) + " |")
    else:
        raise SystemExit("unknown summary kind %r" % kind)
    return 0


def _tuned_large_universe():
    from paper_2003_02842_amd.tune import LARGE_UNIVERSE, load_tuned
    return load_tuned("large-universe") or dict(LARGE_UNIVERSE)


PROFILE_TRAFFIC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic.large-universe.md")


def source_hash(tune=None) -> str:
    """First 16 hex digits of the SHA-256 over the library's kernel sources and
    the plan (mm_tuning dict) the default run uses."""
    import hashlib

    from paper_2003_02842_amd.build import CSRC, HEADERS, SOURCES
    h = hashlib.sha256()
    for f in sorted(SOURCES + HEADERS):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    h.update(repr(sorted((tune or {}).items())).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, tune=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of the default workload, or None when that summary is
    missing or was taken on other kernel sources or another plan."""
    try:
        with open(PROFILE_TRAFFIC) as fh:
            text = fh.read()
    except OSError:
        return None
    tag = "source_sha256_16: "
    if tag not in text or text.split(tag, 1)[1].split()[0] != source_hash(tune):
        return None
    parts = kernel.split("+")
    found = {}
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if cells and cells[0] in parts and len(cells) >= 7:
            found[cells[0]] = float(cells[6])
    return sum(found.values()) if len(found) == len(parts) else None


def copy_calibration():
    import torch
    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
    return 0


def measured_peaks():
    """Reference rates on this device, best of 5: a 2 GiB device-to-device copy
    by torch and by a plain float4 kernel (HBM GB/s, bytes read + written), an
    8192^3 BF16 library GEMM (TFLOP/s) and a loop of back-to-back BF16 MFMAs with
    no memory traffic (TFLOP/s)."""
    import torch
    n = 2 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    a = torch.randn(8192, 8192, device="cuda", dtype=torch.bfloat16)
    b = torch.randn(8192, 8192, device="cuda", dtype=torch.bfloat16)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        t = float("inf")
        for _ in range(5):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t = min(t, e0.elapsed_time(e1))
        return t

    copy_ms = best(lambda: dst.copy_(src))
    gemm_ms = best(lambda: torch.mm(a, b))
    out = {"hbm_copy_gbs": 2 * n / (copy_ms * 1e-3) / 1e9, "bf16_gemm_tflops": 2 * 8192 ** 3 / (gemm_ms * 1e-3) / 1e12}
    # BF16 MFMA issue rate with no memory traffic (libmm_peak.so): 1024 workgroups
    # of four waves, each wave 8 x iters MFMAs of 32 x 32 x 16
    import ctypes
    peak = ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2003_02842_amd", "libmm_peak.so"))
    peak.mm_peak_mfma_bf16.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    blocks, iters = 1024, 4000
    sink = torch.empty(blocks * 256, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def mfma_loop():
        if peak.mm_peak_mfma_bf16(blocks, iters, ctypes.c_void_p(sink.data_ptr()), stream) != 0:
            raise RuntimeError("MFMA peak probe failed to launch")

    mfma_ms = best(mfma_loop)
    out["bf16_mfma_loop_tflops"] = blocks * 4 * iters * 8 * 32768 / (mfma_ms * 1e-3) / 1e12
    # the same 2 GiB copy with a plain float4 kernel, 2048 workgroups
    peak.mm_peak_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]

    def kcopy():
        if peak.mm_peak_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n // 16, 2048,
                             stream) != 0:
            raise RuntimeError("copy probe failed to launch")

    kcopy_ms = best(kcopy)
    out["hbm_copy_kernel_gbs"] = 2 * n / (kcopy_ms * 1e-3) / 1e9
    del src, dst, a, b, sink
    torch.cuda.empty_cache()
    return out


def _timed(fn, steps, warmup):
    import torch
    for _ in range(max(warmup, 1)):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t) / steps


def _best_of(fn, runs):
    """Fastest of `runs` timed calls after one untimed call (ms)."""
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(runs):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, 1e3 * (time.perf_counter() - t))
    return best


def _relfro_max(x, ref):
    """Largest relative Frobenius error over the (cutoff, group) matrices."""
    import torch
    x, ref = x.double(), ref.double()
    fin = torch.isfinite(ref)
    d = torch.where(fin, x - ref, torch.zeros_like(ref))
    r = torch.where(fin, ref, torch.zeros_like(ref))
    return float((torch.linalg.norm(d.flatten(-2), dim=-1) / torch.linalg.norm(r.flatten(-2), dim=-1)).max())


def estimate_bench(a, workload):
    """Monte Carlo replicates (1000 groups of 10 series, 19 cutoffs up to 2000) or
    the 100-asset cross-section (N = 5000), both through mm_estimate (one NUFFT at
    the largest cutoff serves every cutoff), timed as a HIP graph replay and as
    eager launches; `value` takes the faster.  Beside it: the same mixed path
    re-run per cutoff (the loop the paper times), and the plain FP64 form with the
    same reuse.  Accuracy is against the FP64 form at tol 1e-12.  Returns the
    result as a dict."""
    import torch

    from paper_2003_02842_amd import mm, synth

    if workload == "replicates":
        w = synth.epps_replicates(device="cuda")
        G, D, Ns = w.G, w.D, [int(n) for n in w.Ns]
    else:
        w = synth.cross_section().to("cuda")
        G, D, Ns = 1, w.S, [5000]
    torch.cuda.synchronize()
    Nmax, basis, kern, tol = max(Ns), a.basis, a.kernel, a.tol
    ws = torch.empty(mm.estimate_workspace_size(G, D, Ns, kern, tol, "mixed"), dtype=torch.uint8, device="cuda")
    out = (torch.empty((len(Ns), G, D, D), device="cuda"), torch.empty((len(Ns), G, D, D), device="cuda"))

    gst = torch.cuda.Stream()

    def graph_step():
        # replayed on a stream of its own: on torch's default stream the binding
        # would hop to a side stream and back around every replay
        with torch.cuda.stream(gst):
            mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, G, D, Ns, basis, kern, tol, "mixed", out=out, ws=ws,
                        use_graph=True)

    def eager_step():
        mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, G, D, Ns, basis, kern, tol, "mixed", out=out, ws=ws)

    graph_ms = _timed(graph_step, a.steps, a.warmup)
    eager_ms = _timed(eager_step, a.steps, a.warmup)
    ms = min(graph_ms, eager_ms)
    eager_step()
    torch.cuda.synchronize()
    mm.profile_reset()
    mm.profile_enable(True)
    eager_step()
    torch.cuda.synchronize()
    mm.profile_enable(False)
    kern_ms = {}
    for nm in ("k_setup", "k_prep", "k_deconv", "k_fft_tables", "k_tile_ranges", "k_nufft_fused", "k_spread_poly",
               "k_spread_mom", "k_spread", "k_fft_cols_ab",
               "k_fft_rows_ab", "k_cov_small", "k_split_scale", "k_split_bf16", "k_syrk_mfma256", "k_syrk_mfma",
               "k_syrk_reduce", "k_corr"):
        t, n = mm.profile_read(nm)
        if n:
            kern_ms[nm] = round(t / n, 5)

    def per_cutoff():
        for N in Ns:
            c = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, N, kern, tol, "mixed")
            mm.cov(c, G, D, [N], basis)

    plan = mm.plan_query(Nmax, kern, tol, "mixed")
    per_cutoff_ms = plain_ms = errs = None
    if not a.no_plain:
        per_cutoff_ms = _best_of(per_cutoff, 3)
        dp64 = w.dp.double()
        ptune = {"width": plan["width"]}

        def plain():
            c = mm.nufft1(w.offsets, w.t, dp64, w.t0, w.T, Nmax, kern, tol, "fp64", ptune)
            return mm.cov(c, G, D, Ns, basis)

        plain_ms = _best_of(plain, 3)
        S64, R64, _ = mm.estimate(w.offsets, w.t, dp64, w.t0, w.T, G, D, Ns, basis, kern, 1e-12, "fp64")
        graph_step()
        torch.cuda.synchronize()
        errs = {"cov": _relfro_max(out[0], S64), "corr": _relfro_max(out[1], R64)}
    res = {
        "metric": "events/s + contraction TFLOP/s at <=1e-5 rel.err vs FP64; speedup vs plain FP64 GPU",
        "value": w.E / (ms * 1e-3),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16x3" if D * (D + 1) // 2 > 1024 else "f32+f64-sweep",
        "data": "synthetic",
        "config": {"workload": "%s: %d groups x %d series, %d events, cutoffs %s, %s kernel tol %g, %s basis" % (
                       workload, G, D, w.E, Ns if len(Ns) <= 4 else "%d up to %d" % (len(Ns), Nmax), kern, tol,
                       basis), "events": w.E, "series": w.S, "cutoffs": Ns, "width": plan["width"],
                   "Mr": plan["Mr"], "parallelism": "1 GPU"},
        "launch": "graph replay" if graph_ms <= eager_ms else "eager",
        "graph_ms_per_step": graph_ms,
        "eager_ms_per_step": eager_ms,
        "kernels_ms": kern_ms,
        "mixed_rerun_per_cutoff_ms": per_cutoff_ms,
        "plain_fp64_reuse_ms": plain_ms,
        "speedup_vs_plain_fp64": plain_ms / ms if plain_ms else None,
        "speedup_vs_rerun_per_cutoff": per_cutoff_ms / ms if per_cutoff_ms else None,
        "rel_err_vs_fp64": errs,
        "roofline": None,
    }
    del w, ws, out
    torch.cuda.empty_cache()
    return res


def pairwise_bench(a):
    """Per-pair cutoffs N_ij = min(N_i, N_j) on the large universe: every asset with
    its own cutoff (log-spaced over [1000, N], shuffled), mm_cov_pairwise on the
    mixed coefficients (best of 3) beside mm_cov at the single cutoff N and the FP64
    form of the per-pair product; Sigma/R error against that FP64 form."""
    import numpy as np
    import torch

    from paper_2003_02842_amd import mm, synth
    from paper_2003_02842_amd.tune import LARGE_UNIVERSE

    w = synth.large_universe(D=a.D, n_lo=a.n_lo, n_hi=a.n_hi, N=a.N, seed=a.seed, device="cuda")
    D, N = w.S, a.N
    rng = np.random.default_rng(a.seed)
    levels = np.unique(np.round(np.geomspace(1000, N, 4 * D)).astype(int))
    Ni = [int(v) for v in rng.permutation(levels[np.linspace(0, levels.size - 1, D).astype(int)])]
    c = mm.nufft1(w.offsets, w.t, w.dp, w.t0, w.T, N, a.kernel, a.tol, "mixed", dict(LARGE_UNIVERSE))
    ws = torch.empty(max(mm.cov_workspace_size(1, D, N, 1, "mixed"), 256), dtype=torch.uint8, device="cuda")
    pair_ms = _best_of(lambda: mm.cov_pairwise(c, 1, D, Ni, a.basis), 3)
    single_ms = _best_of(lambda: mm.cov(c, 1, D, [N], a.basis, ws=ws), 3)
    S, R = mm.cov_pairwise(c, 1, D, Ni, a.basis)
    # an Epps sweep on the same coefficients: 20 log-spaced cutoffs up to N in one
    # pass over k, beside one product per cutoff
    Ns = sorted({int(v) for v in np.round(np.geomspace(1, N, 20))})
    wsw = torch.empty(max(mm.cov_workspace_size(1, D, N, len(Ns), "mixed"), 256), dtype=torch.uint8, device="cuda")
    sweep_ms = _best_of(lambda: mm.cov(c, 1, D, Ns, a.basis, ws=wsw), 3)
    separate_ms = sum(_best_of(lambda: mm.cov(c, 1, D, [n], a.basis, ws=ws), 3) for n in Ns)
    Sw, Rw = mm.cov(c, 1, D, Ns, a.basis, ws=wsw)
    del c, ws, wsw
    torch.cuda.empty_cache()
    c64 = mm.nufft1(w.offsets, w.t, w.dp.double(), w.t0, w.T, N, a.kernel, 1e-12, "fp64")
    t = time.perf_counter()
    S64, R64 = mm.cov_pairwise(c64, 1, D, Ni, a.basis)
    torch.cuda.synchronize()
    fp64_ms = 1e3 * (time.perf_counter() - t)
    errs = {"cov": _relfro_max(S[None], S64[None]), "corr": _relfro_max(R[None], R64[None])}
    del S, R, S64, R64
    torch.cuda.empty_cache()
    Sw64, Rw64 = mm.cov(c64, 1, D, Ns, a.basis)
    sweep_errs = {"cov": _relfro_max(Sw, Sw64), "corr": _relfro_max(Rw, Rw64)}
    del c64, Sw, Rw, Sw64, Rw64
    torch.cuda.empty_cache()
    return {"ms": pair_ms, "distinct_cutoffs": len(set(Ni)), "cutoff_range": [min(Ni), max(Ni)],
            "single_cutoff_mm_cov_ms": single_ms, "plain_fp64_pairwise_ms": fp64_ms, "rel_err_vs_fp64": errs,
            "config": "large universe, %d assets each with its own cutoff, %s basis, mixed" % (D, a.basis),
            "sweep": {"cutoffs": Ns, "one_pass_ms": sweep_ms, "one_product_per_cutoff_ms": separate_ms,
                      "rel_err_vs_fp64": sweep_errs}}


def main():
    a = parse()
    if a.summarize:
        return summarize(a.summarize)
    if a.copy_calibration:
        return copy_calibration()
    if a.gpus != 1:
        print("bench.py runs on exactly one GPU (the path is single-GPU); --gpus %d is not supported" % a.gpus, file=sys.stderr)
        return 2
    if a.workload == "pairwise":
        print(json.dumps(pairwise_bench(a)), flush=True)
        return 0
    if a.workload != "large-universe":
        print(json.dumps(estimate_bench(a, a.workload)), flush=True)
        return 0
    import torch

    from paper_2003_02842_amd import mm, synth

    dev = "cuda"
    t_gen = time.perf_counter()
    w = synth.large_universe(D=a.D, n_lo=a.n_lo, n_hi=a.n_hi, N=a.N, seed=a.seed, device=dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    E, S, N, D = w.E, w.S, a.N, a.D
    print("# generated %d events in %.1f s" % (E, t_gen), file=sys.stderr, flush=True)

    from paper_2003_02842_amd.tune import LARGE_UNIVERSE, load_tuned
    cached = None if a.untuned else load_tuned("large-universe")
    tune = {} if a.untuned else dict(cached or LARGE_UNIVERSE)
    tune.update({k: v for k, v in (("width", a.width), ("sigma", a.sigma)) if v})
    tune = tune or None
    plan = mm.plan_query(N, a.kernel, a.tol, "mixed", tune)
    wse = torch.empty(mm.estimate_workspace_size(1, D, [N], a.kernel, a.tol, "mixed", tune), dtype=torch.uint8,
                      device=dev)
    res = (torch.empty((1, 1, D, D), device=dev), torch.empty((1, 1, D, D), device=dev))

    def step():
        # both stages in one library call; with no coefficient output the FFT's
        # row pass writes the contraction's BF16 operands itself
        cv, cr, _ = mm.estimate(w.offsets, w.t, w.dp, w.t0, w.T, 1, D, [N], a.basis, a.kernel, a.tol, "mixed", tune,
                                ws=wse, out=res)
        return cv, cr

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    # the timed region: no per-kernel instrumentation
    t0 = time.perf_counter()
    for _ in range(a.steps):
        cov, corr = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # a separate pass with HIP events around every launch (on its stream) for the
    # per-kernel durations of the roofline fields
    mm.profile_reset()
    mm.profile_enable(True)
    for _ in range(max(3, min(a.steps, 10))):
        step()
    torch.cuda.synchronize()
    mm.profile_enable(False)
    # kernel names as launched (the planner picks one kernel per role)
    roles = {"spread": (SPREAD_PAIR, "k_spread_poly", "k_spread"), "fft_cols": ("k_fft_cols_ab", "k_fft_cols"),
             "fft_rows": ("k_fft_rows_ab", "k_fft_rows"), "syrk": ("k_syrk_mfma256", "k_syrk_mfma")}
    names = ["k_setup", "k_prep", "k_deconv", "k_fft_tables", "k_tile_ranges", "k_split_scale", "k_split_pad", "k_split_bf16",
             "k_syrk_reduce", "k_corr", "k_cov_small"] + \
        [n for r in roles.values() for n in r]
    kern = {}
    for nm in names + ["k_spread_mom"]:
        ms, n = mm.profile_read(nm)
        if n:
            kern[nm] = {"avg_ms": ms / n, "launches": n}
    # the spreading pass as two launches splitting the grid tiles between them
    # (per-event taps, per-cell moments): timed and priced as one step
    if "k_spread_mom" in kern and "k_spread_poly" in kern:
        kern[SPREAD_PAIR] = {"avg_ms": kern["k_spread_poly"]["avg_ms"] + kern["k_spread_mom"]["avg_ms"],
                             "launches": kern["k_spread_mom"]["launches"]}
    role = {r: next((n for n in cands if n in kern), None) for r, cands in roles.items()}
    ms_step = 1e3 * elapsed / a.steps
    print("# mixed: %.3f ms/step  %s" % (ms_step, json.dumps({k: round(v["avg_ms"], 4) for k, v in kern.items()})),
          file=sys.stderr, flush=True)

    # the NUFFT's own kernels (mm_nufft1), summed
    t_nufft = sum(kern[k]["avg_ms"] for k in ("k_setup", "k_prep", "k_deconv", "k_fft_tables", "k_tile_ranges",
                                                role["spread"],
                                                role["fft_cols"], role["fft_rows"]) if k in kern)
    # contraction throughput (GEMM-equivalent flops)
    K = 2 * N + 1
    gemm_flops = 2.0 * D * D * K
    t_con = sum(kern[k]["avg_ms"] for k in ("k_split_scale", "k_split_pad", "k_split_bf16", role["syrk"],
                                             "k_syrk_reduce") if k in kern)
    con_tflops = gemm_flops / (t_con * 1e-3) / 1e12 if t_con > 0 else None

    # roofline of the dominant kernel: algorithmic bytes (flops) per launch over the
    # mean launch duration from HIP events on the launch stream
    parts = ("k_spread_poly", "k_spread_mom") if SPREAD_PAIR in kern else ()
    dom = max((k for k in kern if k not in parts), key=lambda k: kern[k]["avg_ms"])
    default_workload = (a.D, a.n_lo, a.n_hi, a.N, a.kernel, a.tol, a.basis, a.seed, a.width, a.sigma, a.untuned) == \
        (2000, 1e4, 1e6, 50_000, "es", 1e-6, "fejer", 20200310, 0, 0.0, False)
    traffic = measured_traffic(dom, tune) if default_workload else None
    Mr = plan["Mr"]
    alg_bytes = {
        role["spread"]: E * (8 + 4) + S * Mr * 4 + (S + 1) * 8,
        role["fft_cols"]: 2 * S * (Mr // 2) * 8,
        role["fft_rows"]: S * (Mr // 2) * 8 + S * (N + 1) * 8,
    }
    Kp = ((2 * (N + 1) + 31) // 32) * 32
    mfma_flops = 3.0 * D * (D + 1) * Kp
    if dom == role["syrk"]:
        ach = mfma_flops / (kern[dom]["avg_ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / BF16_PEAK_TFLOPS, "traffic": traffic}
    else:
        b = alg_bytes.get(dom)
        ach = b / (kern[dom]["avg_ms"] * 1e-3) / 1e9 if b else None
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS if ach else None, "traffic": traffic,
                "alg_bytes": b}
    mfma_t = kern.get(role["syrk"], {}).get("avg_ms")
    contraction_roof = ({"kernel": role["syrk"], "bound": "mfma", "unit": "TFLOP/s", "peak": BF16_PEAK_TFLOPS,
                         "achieved": mfma_flops / (mfma_t * 1e-3) / 1e12,
                         "frac": mfma_flops / (mfma_t * 1e-3) / 1e12 / BF16_PEAK_TFLOPS} if mfma_t else None)
    spread_t = kern.get(role["spread"], {}).get("avg_ms")
    spread_roof = ({"kernel": role["spread"], "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                    "achieved": alg_bytes[role["spread"]] / (spread_t * 1e-3) / 1e9,
                    "frac": alg_bytes[role["spread"]] / (spread_t * 1e-3) / 1e9 / HBM_PEAK_GBS} if spread_t else None)

    out = {
        "metric": "events/s + contraction TFLOP/s at <=1e-5 rel.err vs FP64; speedup vs plain FP64 GPU",
        "value": E * a.steps / elapsed,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16x3",
        "data": "synthetic",
        "config": {"workload": "large-universe: D=%d 3-factor GBM, log-uniform counts [%g, %g], T=28800 s, N=%d, "
                               "%s kernel, %s basis" % (D, a.n_lo, a.n_hi, N, a.kernel, a.basis),
                   "events": E, "series": S, "N": N, "tol": a.tol, "width": plan["width"], "sigma": plan["sigma"], "Mr": Mr,
                   "tuning": tune, "tuning_source": ("none" if a.untuned else
                                                     "tuned_plans.json" if cached else "built-in default"),
                   "seed": a.seed, "parallelism": "1 GPU"},
        "nufft1_ms": t_nufft,
        "nufft1_events_per_s": E / (t_nufft * 1e-3) if t_nufft else None,
        "contraction_tflops": con_tflops,
        "kernels_ms": {k: round(v["avg_ms"], 5) for k, v in kern.items()},
        "roofline": roof,
        "roofline_spread": spread_roof,
        "roofline_contraction": contraction_roof,
        "measured_peaks": measured_peaks(),
    }

    # plain FP64 GPU form on the same input with the same kernel width (so the same
    # accuracy), one launch chain per series and the FP64 contraction
    if not a.no_plain:
        dp64 = w.dp.to(torch.float64)
        coef64 = torch.empty((S, N + 1), dtype=torch.complex128, device=dev)
        ptune = {"width": plan["width"], "sigma": plan["sigma"]}
        wsp = torch.empty(mm.nufft1_workspace_size(S, N, a.kernel, a.tol, "fp64", ptune), dtype=torch.uint8,
                          device=dev)

        def plain_step():
            mm.nufft1(w.offsets, w.t, dp64, w.t0, w.T, N, a.kernel, a.tol, "fp64", ptune, out=coef64, ws=wsp)
            return mm.cov(coef64, 1, D, [N], a.basis)

        plain_ms = _best_of(plain_step, 3)
        out["plain_fp64_ms_per_step"] = plain_ms
        out["plain_fp64_width"] = plan["width"]
        out["speedup_vs_plain_fp64"] = plain_ms / ms_step
        # reference for the error: FP64 GPU form at tol 1e-12
        wsr = torch.empty(mm.nufft1_workspace_size(S, N, a.kernel, 1e-12, "fp64"), dtype=torch.uint8, device=dev)
        mm.nufft1(w.offsets, w.t, dp64, w.t0, w.T, N, a.kernel, 1e-12, "fp64", out=coef64, ws=wsr)
        c64, r64 = mm.cov(coef64, 1, D, [N], a.basis)
        cov_err = float(torch.linalg.norm((cov.double() - c64).flatten()) / torch.linalg.norm(c64.flatten()))
        fin = torch.isfinite(r64)
        corr_err = float(torch.linalg.norm((corr.double() - r64)[fin]) / torch.linalg.norm(r64[fin]))
        out["rel_err_vs_fp64"] = {"cov": cov_err, "corr": corr_err}
        del dp64, coef64, wsp, wsr

    # CPU oracle on a bounded, count-stratified sample of the same workload: ten
    # series from the smallest to the densest, every stride-th k; the direct sum's
    # cost is exactly linear in (events x k), so the rate over all k = 0..N follows
    # by scaling; fastest of three runs
    if not a.no_cpu:
        import numpy as np

        import oracle

        counts = (w.offsets[1:] - w.offsets[:-1]).cpu()
        order = torch.argsort(counts).tolist()
        picks = sorted({order[(q * (len(order) - 1)) // 9] for q in range(10)})
        sub = w.subset(picks).to("cpu")
        tts = [sub.series(i) for i in range(len(picks))]

        def run(ks):
            t1 = time.perf_counter()
            for tt, dd in tts:
                oracle.coeffs_at(tt, dd, sub.t0, sub.T, ks)
            return time.perf_counter() - t1

        probe = np.arange(0, N + 1, max(1, (N + 1) // 16), dtype=np.int64)
        run(probe)   # the first call starts the oracle's threads
        per_k = run(probe) / probe.size
        stride = max(1, int(math.ceil((N + 1) * per_k / max(a.cpu_seconds / 3.0, 1e-3))))
        ks = np.arange(0, N + 1, stride, dtype=np.int64)
        best = min(run(ks) for _ in range(3))
        rate = sub.E * (ks.size / (N + 1)) / best
        out["cpu_baseline"] = {"value": rate, "unit": "events/s", "cores": oracle.threads(), "kind": "oracle",
                               "sample": "%d series stratified over the count range (%d to %d events, %d in all), "
                                         "coefficients at every %d-th k of 0..%d (%d values), fastest of 3 runs "
                                         "(%.2f s); scaled to all N+1 = %d coefficients per event, which the direct "
                                         "sum costs in proportion" % (len(picks), int(counts[picks].min()),
                                                                      int(counts[picks].max()), sub.E, stride, N,
                                                                      ks.size, best, N + 1)}
    # the other two workloads through mm_estimate (C3 cross-section, C4 replicates)
    if not a.no_extra:
        del w, wse, res, cov, corr
        torch.cuda.empty_cache()
        ea = argparse.Namespace(**vars(a))
        ea.steps, ea.warmup = max(10, a.steps), 3
        for name in ("cross-section", "replicates"):
            r = estimate_bench(ea, name)
            out[name.replace("-", "_")] = {k: r[k] for k in (
                "value", "unit", "ms_per_step", "launch", "graph_ms_per_step", "eager_ms_per_step", "kernels_ms",
                "mixed_rerun_per_cutoff_ms", "plain_fp64_reuse_ms", "speedup_vs_plain_fp64",
                "speedup_vs_rerun_per_cutoff", "rel_err_vs_fp64", "config", "dtype")}
        out["pairwise"] = pairwise_bench(ea)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
