"""Comparison rules between the GPU path and the FP64 oracle.

Correlation: per pair-frame, e = max_i |y_gpu - y_ref| / max_i |y_ref|; pair-frames
whose reference is identically zero are left out.

Integer TDoA: must match exactly wherever the reference's two largest values
(at any lags) differ by more than 2 * eps * max|y_ref|: an entry-wise error of
at most eps * max|y_ref| cannot move the argmax there.  Elsewhere several
answers are within rounding of the maximum, and the GPU's answer must be one
of them.
"""
from __future__ import annotations

import numpy as np


def corr_errors(y_gpu, y_ref):
    y_gpu = np.asarray(y_gpu, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    scale = np.abs(y_ref).max(-1)
    err = np.abs(y_gpu - y_ref).max(-1)
    ok = scale > 0
    return err[ok] / scale[ok]


def tdoa_report(t_gpu, y_ref, tau_max: int, eps: float) -> dict:
    y_ref = np.asarray(y_ref, dtype=np.float64)
    t_gpu = np.asarray(t_gpu)
    t_ref = np.argmax(y_ref, axis=-1) - tau_max
    s = np.sort(y_ref, axis=-1)
    scale = np.abs(y_ref).max(-1)
    gap = s[..., -1] - s[..., -2] if y_ref.shape[-1] > 1 else scale
    qualified = (gap > 2.0 * eps * scale) & (scale > 0)
    # where not qualified, the GPU's lag must be within 2 eps scale of the max
    idx = np.clip(t_gpu + tau_max, 0, y_ref.shape[-1] - 1)
    val = np.take_along_axis(y_ref, idx[..., None], axis=-1)[..., 0]
    near_max = val >= s[..., -1] - 2.0 * eps * scale
    in_range = (t_gpu >= -tau_max) & (t_gpu <= tau_max)
    return {
        "n": int(t_gpu.size),
        "qualified": int(qualified.sum()),
        "mismatch_qualified": int((qualified & (t_gpu != t_ref)).sum()),
        "agreement": float((t_gpu == t_ref).mean()) if t_gpu.size else 1.0,
        "agreement_qualified": float((t_gpu == t_ref)[qualified].mean()) if qualified.any() else 1.0,
        "invalid_elsewhere": int((~qualified & ~(near_max & in_range)).sum()),
    }
