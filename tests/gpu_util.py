"""Helpers shared by the GPU tests: upload synthetic frames and compare the
HIP path with the oracle at the stated bar."""
from __future__ import annotations

import numpy as np

FEATURE_RTOL = 1e-5   # relative bound on E, h and L against the FP64 oracle


def to_device(video, device="cuda"):
    """Uploads planes; 10-bit samples travel as int16 (same bytes as uint16)."""
    import torch
    out = []
    for p in (video.y, video.u, video.v):
        a = np.ascontiguousarray(p)
        if a.dtype == np.uint16:
            a = a.view(np.int16)
        out.append(torch.from_numpy(a).to(device))
    return tuple(out)


def assert_features_close(gpu: np.ndarray, ref: np.ndarray, rtol: float = FEATURE_RTOL):
    """Relative error <= rtol everywhere; exact 0.0 where the oracle gives 0."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    zero = ref == 0.0
    assert (gpu[zero] == 0.0).all(), f"nonzero where oracle is 0: {gpu[zero]}"
    nz = ~zero
    rel = np.abs(gpu[nz] - ref[nz]) / np.abs(ref[nz])
    worst = rel.max() if rel.size else 0.0
    assert worst <= rtol, f"max relative feature error {worst:.3e} > {rtol:.0e}"
    return worst


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
