"""Per-camera-stream frame loop over the C ABI (Sec. 2: disparity prediction,
stereo matching in the reduced space, disparity update).

A StreamState keeps the stream's disparity and variance maps resident on the
GPU between frames together with every buffer a frame needs, so a frame
enqueues only kernels.  Frame 0, and every frame after reset(), matches over
the full range; later frames warp the previous map by the ego-motion, refine
the prediction (edge rejection and hole filling, Sec. 2.2.2), derive per-pixel
windows from the predicted variance (or a fixed radius) and match only inside
them (Sec. 2.3; Sec. 3: the first frame searches everything).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import egosgm as eg


@dataclass
class Calib:
    f: float
    cx: float
    cy: float
    baseline: float


@dataclass
class FrameConfig:
    max_disp: int = 128
    p1: int = 10
    p2: int = 120
    s_max: int = 80
    lr_tol: int = 1
    q: float = 0.5            # ego-motion variance in disparity space (Eq. 5)
    k_sigma: float = 3.0      # window half-width in standard deviations (Sec. 2.3)
    r_fixed: int = -1         # >= 0: fixed window radius instead of k_sigma*sqrt(p)
    r_min: int = 0
    r_max: int = 256
    keep_unmeasured: int = 0
    edge_tol: float = 2.0     # prediction edge rejection (Sec. 2.2.2); < 0 disables
    fill_tol: float = 1.0     # one-pixel hole filling, Eq. 7-8; <= 0 disables
    full_range_only: bool = False   # plain SGM every frame (the baseline)
    n_paths: int = 8          # 4: the cheaper variant along rows and columns only
    sad_radius: int = 0       # > 0: SAD check on (2r+1)^2 patches after matching (Sec. 2.4.1)
    sad_max: int = 600
    lr_predict: bool = False  # left-right check of the prediction against the warped right map
    lr_predict_tol: float = 1.0
    overlap_census: bool = False  # step(): census on a second stream (measured 2% slower here)
    vo: bool = False          # step(): ego-motion from the images (estimate_motion) instead of R, t given
    vo_levels: int = 0        # pyramid levels (0: the coarsest level stays >= 64 x 16)
    # Gauss-Newton iterations per level, finest first, starting from the previous frame's motion
    # (more gave the same poses on the street sequences), and without one to start from
    vo_iters: tuple = (1, 2, 2, 2, 2, 2)
    vo_iters_first: tuple = (2, 4, 8, 10, 20, 30)
    vo_huber: float = 8.0
    vo_min_disp: float = 1.0

    def match(self) -> eg.MatchParams:
        return eg.MatchParams(self.max_disp, self.p1, self.p2, self.s_max, self.lr_tol,
                              self.n_paths)


class StreamState:
    """own_matcher=False: the stream is matched through a batched plan (no
    matcher workspace or outputs of its own; update() takes the plan's)."""

    def __init__(self, w: int, h: int, calib: Calib, cfg: FrameConfig, device="cuda",
                 own_matcher: bool = True):
        self.w, self.h, self.calib, self.cfg = w, h, calib, cfg
        dev = torch.device(device)
        self.device = dev
        n = w * h
        f32 = dict(dtype=torch.float32, device=dev)
        self.d = torch.full((h, w), -1.0, **f32)     # D^{k}
        self.p = torch.zeros((h, w), **f32)          # P^{k}
        self.d_pred = torch.empty((h, w), **f32)
        self.p_pred = torch.empty((h, w), **f32)
        self.zbuf = torch.empty(n, dtype=torch.int64, device=dev)
        self.lo = torch.empty((h, w), dtype=torch.int16, device=dev)
        self.hi = torch.empty((h, w), dtype=torch.int16, device=dev)
        self.off = torch.empty(n + 1, dtype=torch.int32, device=dev)
        self.out = dict(disp_wta=torch.empty((h, w), dtype=torch.int16, device=dev),
                        disp_sub=torch.empty((h, w), **f32),
                        var_meas=torch.empty((h, w), **f32),
                        disp_right=torch.empty((h, w), dtype=torch.int16, device=dev)) \
            if own_matcher else {}
        self.ws = eg.Workspace(dev)
        if own_matcher:
            self.ws.sgm_bytes(w, h, cfg.max_disp)
        self.ws.windows_bytes(w, h)
        self.ws.refine_bytes(w, h)
        self.invalid = torch.full((h, w), -1.0, **f32)
        self.zeros = torch.zeros((h, w), **f32)
        # step() runs the matcher's census on a second stream (default
        # priority) while the prediction of the frame runs on the caller's
        self.side = torch.cuda.Stream(device=dev) if own_matcher and cfg.overlap_census else None
        self.ev_census = torch.cuda.Event() if self.side is not None else None
        self.census_pending = False
        if cfg.lr_predict:   # right map of the previous frame and its prediction
            self.d_r = torch.full((h, w), -1.0, **f32)
            self.d_rwarp = torch.empty((h, w), **f32)
            self.p_rwarp = torch.empty((h, w), **f32)
            self.d_rpred = torch.empty((h, w), **f32)
            self.p_rpred = torch.empty((h, w), **f32)
        if cfg.vo:   # previous left image, the motion estimate (kept as the next guess)
            levels = cfg.vo_levels or eg.vo_levels_for(w, h)
            self.vo_prm = eg.vo_params(levels, cfg.vo_iters[:levels], cfg.vo_huber, cfg.vo_min_disp)
            self.vo_prm_first = eg.vo_params(levels, cfg.vo_iters_first[:levels], cfg.vo_huber, cfg.vo_min_disp)
            self.vo_ws = eg.vo_workspace(w, h, self.vo_prm, dev)
            self.prev_left = torch.empty((h, w), dtype=torch.uint8, device=dev)
            self.vo_pose = torch.zeros(12, dtype=torch.float64, device=dev)
            self.vo_motion = None
        self.frame = 0

    def reset(self):
        """Drop the prediction: the next frame searches the full range."""
        self.frame = 0
        if self.cfg.vo:
            self.vo_motion = None

    def full_range_next(self) -> bool:
        return self.frame == 0 or self.cfg.full_range_only

    def predict(self, R=None, t=None):
        """First half of a frame: warp, refine and windows (Sec. 2.2-2.3).
        Returns (lo, hi, offsets) for this frame, or None when it is matched
        over the full range."""
        if self.full_range_next():
            return None
        cfg, c = self.cfg, self.calib
        # warp (Sec. 2.2) and refinement (Sec. 2.2.2), fused: the refinement
        # decodes the warp's z-buffer itself
        eg.predict_disparity(self.d, self.p, R, t, c.f, c.cx, c.cy, c.baseline, cfg.q,
                             cfg.edge_tol, cfg.fill_tol, out=(self.d_pred, self.p_pred),
                             zbuf=self.zbuf)
        if cfg.lr_predict:
            # Fig. 4 (d): the right map is predicted the same way, with the
            # right camera's motion, and the left prediction checked against it
            Rr, tr = eg.right_motion(R, t, c.baseline)
            eg.warp_disparity(self.d_r, self.zeros, Rr, tr, c.f, c.cx, c.cy, c.baseline, cfg.q,
                              out=(self.d_rwarp, self.p_rwarp), zbuf=self.zbuf)
            eg.refine_prediction(self.d_rwarp, self.p_rwarp, cfg.edge_tol, cfg.fill_tol,
                                 out=(self.d_rpred, self.p_rpred), workspace=self.ws)
            eg.lr_check_prediction(self.d_pred, self.p_pred, self.d_rpred, cfg.lr_predict_tol)
        eg.windows_from_prediction(self.d_pred, self.p_pred, cfg.max_disp, cfg.r_fixed,
                                   cfg.r_min, cfg.r_max, cfg.k_sigma,
                                   out=(self.lo, self.hi, self.off), workspace=self.ws)
        return self.lo, self.hi, self.off

    def census_ahead(self, left: torch.Tensor, right: torch.Tensor):
        """Starts the matcher's census pass of this frame on the second
        stream, after the previous frame's matcher is done with the
        workspace; match() then waits for it and skips its own."""
        # after everything enqueued on the caller's stream so far: the
        # previous frame's matcher (done with the workspace) and whatever
        # produced the images (an asynchronous copy, a renderer)
        self.side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.side):
            eg.sgm_census(left, right, self.cfg.max_disp, workspace=self.ws)
            self.ev_census.record(self.side)
        left.record_stream(self.side)    # the allocator must not hand them out before
        right.record_stream(self.side)   # the side stream is done with them
        self.census_pending = True

    def match(self, left: torch.Tensor, right: torch.Tensor, windows):
        """Stereo matching of this frame into self.out (Sec. 2.3)."""
        prm = self.cfg.match()
        if self.census_pending:
            torch.cuda.current_stream(self.device).wait_event(self.ev_census)
            prm.census_ready = 1
            self.census_pending = False
        if windows is None:
            eg.sgm_full(left, right, prm, out=self.out, workspace=self.ws)
        else:
            eg.sgm_reduced(left, right, *windows, prm, out=self.out, workspace=self.ws)
        self.filter(left, right, self.out)

    def filter(self, left, right, out):
        """Outlier filters after matching besides the left-right check."""
        if self.cfg.sad_radius > 0:
            eg.sad_check(left, right, out, self.cfg.sad_radius, self.cfg.sad_max)

    def update(self, out=None):
        """Second half: the Kalman update of the prediction with the
        measurement (self.out, or the outputs dict `out` of a batched plan)
        (Sec. 2.4); the first frame takes the measurement as it is."""
        cfg = self.cfg
        out = out or self.out
        if self.full_range_next():
            eg.kalman_update(self.invalid, self.zeros, out["disp_sub"], out["var_meas"],
                             cfg.keep_unmeasured, out=(self.d, self.p))
        else:
            eg.kalman_update(self.d_pred, self.p_pred, out["disp_sub"], out["var_meas"],
                             cfg.keep_unmeasured, out=(self.d, self.p))
        if cfg.lr_predict:
            eg.disparity_to_float(out["disp_right"], self.d_r)
        self.frame += 1
        return self.d, self.p

    def resident_bytes(self) -> int:
        """Device bytes this stream holds (maps, prediction buffers, windows,
        outputs and workspaces)."""
        ts = [self.d, self.p, self.d_pred, self.p_pred, self.zbuf,
              self.lo, self.hi, self.off, self.invalid, self.zeros, *self.out.values(),
              *[getattr(self, k, None) for k in ("d_r", "d_rwarp", "p_rwarp", "d_rpred", "p_rpred")],
              self.ws.sgm, self.ws.win, getattr(self.ws, "ref", None),
              *[getattr(self, k, None) for k in ("vo_ws", "prev_left", "vo_pose")]]
        return sum(t.numel() * t.element_size() for t in ts if t is not None)

    def estimate_motion(self, left: torch.Tensor):
        """Ego-motion from the previous left image and disparity map to this
        left image (estimate_motion), starting from the previous frame's
        estimate; reads the result to the host (a synchronisation), since the
        warp takes the motion as host values."""
        first = self.vo_motion is None
        if first:   # no previous estimate: start at rest, with more iterations on the coarse levels
            self.vo_pose.copy_(torch.tensor(np.concatenate([np.eye(3).ravel(), np.zeros(3)]),
                                            dtype=torch.float64))
        c = self.calib
        eg.estimate_motion(self.prev_left, left, self.d, (c.f, c.cx, c.cy, c.baseline),
                           self.vo_prm_first if first else self.vo_prm, pose=self.vo_pose, workspace=self.vo_ws)
        self.vo_motion = eg.pose_to_host(self.vo_pose)
        return self.vo_motion

    def step(self, left: torch.Tensor, right: torch.Tensor, R=None, t=None):
        """Processes one stereo frame; R, t map the previous camera frame to
        this one (M_k = R M_{k-1} + t); with FrameConfig.vo they are
        estimated from the images instead.  Returns the updated (d, p) maps."""
        if self.cfg.vo and not self.full_range_next():
            R, t = self.estimate_motion(left)
        if self.side is not None:
            self.census_ahead(left, right)
        win = self.predict(R, t)
        self.match(left, right, win)
        if self.cfg.vo:
            self.prev_left.copy_(left)
        return self.update()

    def searched_slots(self) -> int:
        """Disparities searched by the last reduced frame (synchronises)."""
        return int(self.off[self.w * self.h].item()) & 0xFFFFFFFF


def camera_of(seq) -> Calib:
    cam = seq.cam
    return Calib(cam.f, cam.cx, cam.cy, cam.baseline)


def motions(seq):
    return [None] + [tuple(np.asarray(a, np.float64) for a in seq.motion(k))
                     for k in range(1, seq.n_frames)]
