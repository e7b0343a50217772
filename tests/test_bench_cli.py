"""bench.py's command-line contract that needs no GPU: any GPU count other than one,
and any unknown workload, is refused with a message and exit status 2, before
anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_unknown_workload_is_rejected():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "no-such-workload"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr


def test_mfma_peak_probe_is_built():
    """bench.py's measured MFMA ceiling comes from libmm_peak.so (no GPU call here)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2003_02842_amd", "libmm_peak.so"))
    assert hasattr(lib, "mm_peak_mfma_bf16")
