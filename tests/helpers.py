"""Shared helpers of the GPU parity tests (comparison metrics, device checks)."""
import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_02842_amd import mm
    mm.lib()   # raises if the HIP library is missing: no fallback path exists


def relfro(a, b):
    """Relative Frobenius error ||a - b|| / ||b|| over entries finite in b; the
    NaN pattern of a must equal b's."""
    a = np.asarray(a.detach().cpu() if hasattr(a, "detach") else a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    fa, fb = np.isfinite(a), np.isfinite(b)
    assert np.array_equal(fa, fb), "non-finite pattern differs"
    nb = np.linalg.norm(b[fb])
    if nb == 0:
        return float(np.linalg.norm(a[fa]))
    return float(np.linalg.norm(a[fa] - b[fb]) / nb)


def series_rel_l2(coef_gpu, coef_ref):
    """Per-series relative l2 error of the coefficient vectors (Eq. Der:18)."""
    a = coef_gpu.detach().cpu().numpy() if hasattr(coef_gpu, "detach") else coef_gpu
    out = []
    for s in range(coef_ref.shape[0]):
        n = np.linalg.norm(coef_ref[s])
        out.append(np.linalg.norm(a[s, :coef_ref.shape[1]] - coef_ref[s]) / n if n > 0 else np.linalg.norm(a[s]))
    return np.array(out)
