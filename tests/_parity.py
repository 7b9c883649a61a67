"""Comparison helpers for GPU-vs-oracle parity (tolerances and their derivation).

Times and slews: |gpu - ref| <= max(1e-4 |ref|, 1e-3 ps), infinities equal in sign.
Slack is a difference of a required and an arrival time, each held to that bound, so its
bound is max(1e-4 (|RAT| + |AT|), 1e-3 ps).
"""
from __future__ import annotations

import numpy as np


def time_errors(gpu, ref, scale=None, rel=1e-4, abs_=1e-3):
    """Returns (n_bad, worst_ratio, mask_bad) for float times against float64 references."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    inf_r = np.isinf(ref)
    inf_ok = np.array_equal(np.isinf(gpu), inf_r) and np.array_equal(np.sign(gpu[inf_r]), np.sign(ref[inf_r]))
    fin = ~inf_r
    mag = np.abs(ref) if scale is None else np.asarray(scale, np.float64)
    tol = np.maximum(rel * mag, abs_)
    err = np.where(fin, np.abs(gpu - np.where(fin, ref, 0.0)), 0.0)
    ratio = np.where(fin, err / tol, 0.0)
    bad = (ratio > 1.0) | np.isnan(gpu) & fin
    if not inf_ok:
        bad = bad | (np.isinf(gpu) != inf_r)
    return int(bad.sum()), float(np.nanmax(ratio)) if ratio.size else 0.0, bad


def assert_times(gpu, ref, what, scale=None):
    n, worst, _ = time_errors(gpu, ref, scale)
    assert n == 0, f"{what}: {n} values outside tolerance (worst {worst:.3g}x tolerance)"
    return worst


def grad_stats(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    diff = np.abs(gpu - ref)
    gmax = np.abs(ref).max() if ref.size else 0.0
    rel = diff / np.maximum(np.abs(ref), 1e-300)
    norm = np.linalg.norm(gpu - ref) / max(np.linalg.norm(ref), 1e-300)
    return dict(norm_rel=float(norm), gmax=float(gmax), max_abs=float(diff.max()),
                p99_rel=float(np.quantile(rel[np.abs(ref) > 1e-6 * gmax], 0.99)) if gmax > 0 else 0.0,
                max_rel_big=float(rel[np.abs(ref) > 1e-3 * gmax].max()) if gmax > 0 else 0.0)
