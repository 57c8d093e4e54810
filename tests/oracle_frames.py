"""One frame of the method of Sec. 2 on the CPU oracle (test infrastructure).

A frame takes the previous maps D^{k-1}, P^{k-1} and the ego-motion (R, t),
predicts the map (warp, Sec. 2.2, Eq. 1-6, and the refinement of Sec.
2.2.2), derives the search windows (Sec. 2.3), matches inside them (Sec.
2.3-2.4.1) and fuses prediction and measurement (Sec. 2.4, Eq. 10-12).  The
first frame (no previous map) is matched over the full range and takes the
measurement as it is.  Every step is an oracle call; this module only
chains them, so the GPU tests can compare each intermediate result.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc


def predict(d_prev, p_prev, R, t, calib, cfg):
    """Warp and refinement: float32 (d_pred, p_pred) and the warp's winners."""
    wp = orc.warp(np.asarray(d_prev, np.float32), np.asarray(p_prev, np.float32), R, t,
                  calib.f, calib.cx, calib.cy, calib.baseline, cfg.q)
    d, p = orc.refine(wp["d_pred"].astype(np.float32), wp["p_pred"].astype(np.float32),
                      cfg.edge_tol, cfg.fill_tol)
    return d, p, wp


def windows(d_pred, p_pred, cfg):
    return orc.windows(d_pred, p_pred, cfg.max_disp, r_fixed=cfg.r_fixed, r_min=cfg.r_min,
                       r_max=cfg.r_max, k_sigma=cfg.k_sigma)


def match(left, right, cfg, win=None):
    return orc.sgm(left, right, cfg.max_disp, cfg.p1, cfg.p2, cfg.s_max, cfg.lr_tol,
                   windows=win, n_paths=cfg.n_paths)


def update(d_pred, p_pred, o, cfg):
    """Kalman update with the float32 measurement; d_pred None = first frame."""
    z = o["disp_sub"].astype(np.float32)
    r = o["var_meas"].astype(np.float32)
    if d_pred is None:
        shape = z.shape
        return orc.kalman(np.full(shape, -1, np.float32), np.zeros(shape, np.float32), z, r)
    return orc.kalman(d_pred, p_pred, z, r, cfg.keep_unmeasured)


def frame(left, right, d_prev, p_prev, motion, calib, cfg):
    """One frame; d_prev None (or motion None) matches over the full range.
    Returns dict with d_pred, p_pred, win (None for the full range), sgm
    (the matcher's outputs) and d, p (float64 values of the update)."""
    left = np.asarray(left, np.uint8)
    right = np.asarray(right, np.uint8)
    if d_prev is None or motion is None:
        o = match(left, right, cfg)
        d, p = update(None, None, o, cfg)
        return dict(d_pred=None, p_pred=None, win=None, sgm=o, d=d, p=p)
    dp, pp, _ = predict(d_prev, p_prev, motion[0], motion[1], calib, cfg)
    win = windows(dp, pp, cfg)
    o = match(left, right, cfg, win)
    d, p = update(dp, pp, o, cfg)
    return dict(d_pred=dp, p_pred=pp, win=win, sgm=o, d=d, p=p)
