"""Disparity quality against ground truth (the evaluation of Sec. 3).

The paper scores a map by its bad-pixel rate: a pixel is bad when its
disparity error exceeds 3 px or 5% of the true disparity (the paper words
the two thresholds with "or"; KITTI's D1 metric requires both, so both are
reported).  Pixels without an estimate count as bad in the all-pixel rate
and are left out of the estimated-pixel rate; density is the fraction of
evaluated pixels that have an estimate.  Evaluated pixels are those whose
true disparity lies in [0, max_disp).
"""
from __future__ import annotations

import numpy as np


def bad_pixels(d, gt, max_disp: int, abs_px: float = 3.0, rel: float = 0.05) -> dict:
    """d: estimated disparity (any negative value = no estimate), gt: true
    disparity, same shape (numpy arrays or torch tensors)."""
    d = d.detach().cpu().numpy() if hasattr(d, "detach") else np.asarray(d)
    gt = gt.detach().cpu().numpy() if hasattr(gt, "detach") else np.asarray(gt)
    d = d.astype(np.float64)
    gt = gt.astype(np.float64)
    ev = np.isfinite(gt) & (gt >= 0) & (gt < max_disp)
    est = ev & (d >= 0)
    err = np.abs(d - gt)
    big_abs, big_rel = err > abs_px, err > rel * gt
    n, n_est = int(ev.sum()), int(est.sum())

    def rate(bad, over_all):
        b = int((bad & est).sum())
        return (b + (n - n_est) if over_all else b) / max(over_all and n or n_est, 1)

    return {
        "n": n,
        "density": n_est / max(n, 1),
        "bad_or_all": rate(big_abs | big_rel, True),
        "bad_and_all": rate(big_abs & big_rel, True),
        "bad_or_est": rate(big_abs | big_rel, False),
        "bad_and_est": rate(big_abs & big_rel, False),
    }


def summarise(per_frame: list[dict]) -> dict:
    """Means over frames of every rate in per_frame."""
    keys = [k for k in per_frame[0] if k != "n"]
    return {k: round(float(np.mean([f[k] for f in per_frame])), 4) for k in keys}
