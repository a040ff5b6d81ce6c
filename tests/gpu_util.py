"""Shared helpers of the GPU parity tests (comparison metrics and test inputs)."""
from __future__ import annotations

import numpy as np

from paper_1201_2025_amd import synth


def scene(seed, H, W, L, K=4, n_single=None, n_blob=0):
    if n_single is None:
        n_single = max(1, H * W // 400)
    return synth.make_scene(seed, H, W, L, K=K, n_single=n_single, n_blob=n_blob)


def dwt_rel_err(a, ref):
    """Per-pixel normwise relative error max_k |a - ref| / max_k |ref| (max over pixels)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, ref.shape[-1])
    r = np.asarray(ref, dtype=np.float64).reshape(-1, ref.shape[-1])
    num = np.abs(a - r).max(axis=1)
    den = np.maximum(np.abs(r).max(axis=1), 1e-30)
    return float((num / den).max())


def score_rel_err(s, ref, floor_rel=1e-3):
    """Elementwise relative error with a floor of floor_rel * median(|ref|).  Returns the
    error array (non-finite positions must match and count as 0)."""
    s = np.asarray(s, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    fin = np.isfinite(r)
    assert np.array_equal(fin, np.isfinite(s)), "non-finite positions differ"
    assert np.array_equal(np.isnan(r), np.isnan(s)), "NaN positions differ"
    err = np.zeros_like(r)
    if fin.any():
        floor = floor_rel * np.median(np.abs(r[fin]))
        den = np.maximum(np.abs(r[fin]), max(floor, 1e-300))
        err[fin] = np.abs(s[fin] - r[fin]) / den
    return err


def err_summary(err):
    e = np.asarray(err)
    return "max %.3g p99 %.3g median %.3g" % (e.max(), np.percentile(e, 99), np.median(e))


def sample_pixels(H, W, n, seed=0, border=True):
    """n distinct flat pixel indices; includes the four corners and edge pixels."""
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(H * W, size=min(n, H * W), replace=False).tolist())
    if border:
        for y, x in [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, 0), (0, W // 2),
                     (H - 1, W // 2), (H // 2, W - 1), (H // 2, W // 2)]:
            idx.add(y * W + x)
    return np.array(sorted(idx), dtype=np.int64)
