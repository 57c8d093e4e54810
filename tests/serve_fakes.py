"""A CPU executor for the serving scheduler, backed by the oracle (test
infrastructure: it runs the method of Sec. 2 per stream with the plain C
oracle, so the scheduler's admission, ordering and failure handling can be
tested without a GPU)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc
from paper_1708_06301_amd.serve import StreamFailed


class OracleExecutor:
    def __init__(self, n_slots: int = 2, polls_until_done: int = 1, bytes_per_pixel: int = 100):
        self.n_slots = n_slots
        self.polls = polls_until_done
        self.bpp = bytes_per_pixel
        self.streams = {}
        self.fail = set()            # (sid, seq) pairs whose launch raises
        self.launches = []           # [(sid, seq, full_range)] per launch
        self.busy = 0

    def reserve_bytes(self, spec) -> int:
        return spec.w * spec.h * self.bpp

    def open(self, sid, spec):
        self.streams[sid] = dict(spec=spec, d=None, p=None)

    def close(self, sid):
        self.streams.pop(sid)

    def launch(self, group):
        if self.busy >= self.n_slots:
            raise AssertionError("more launches in flight than slots")
        for r in group:
            if r.sid not in self.streams:
                raise AssertionError(f"launch of a closed stream {r.sid}")
            if (r.sid, r.seq) in self.fail:
                raise StreamFailed(r.sid, "forced error")
        outs, rec = [], []
        for r in group:
            e = self.streams[r.sid]
            spec, cfg = e["spec"], e["spec"].cfg
            c = spec.calib
            L, R = np.asarray(r.left), np.asarray(r.right)
            full = r.reset or e["d"] is None
            if full:
                o = orc.sgm(L, R, cfg.max_disp, cfg.p1, cfg.p2, cfg.s_max, cfg.lr_tol)
                dk, pk = orc.kalman(np.full(L.shape, -1, np.float32), np.zeros(L.shape, np.float32),
                                    o["disp_sub"].astype(np.float32),
                                    o["var_meas"].astype(np.float32))
            else:
                wp = orc.warp(e["d"], e["p"], r.R, r.t, c.f, c.cx, c.cy, c.baseline, cfg.q)
                dp, pp = orc.refine(wp["d_pred"].astype(np.float32),
                                    wp["p_pred"].astype(np.float32), cfg.edge_tol, cfg.fill_tol)
                win = orc.windows(dp, pp, cfg.max_disp, r_fixed=cfg.r_fixed, r_min=cfg.r_min,
                                  r_max=cfg.r_max, k_sigma=cfg.k_sigma)
                o = orc.sgm(L, R, cfg.max_disp, cfg.p1, cfg.p2, cfg.s_max, cfg.lr_tol, windows=win)
                dk, pk = orc.kalman(dp, pp, o["disp_sub"].astype(np.float32),
                                    o["var_meas"].astype(np.float32), cfg.keep_unmeasured)
            e["d"], e["p"] = dk.astype(np.float32), pk.astype(np.float32)
            outs.append(dict(full_range=full, d=e["d"].copy(), p=e["p"].copy()))
            rec.append((r.sid, r.seq, full))
        self.launches.append(rec)
        self.busy += 1
        return dict(outs=outs, polls=self.polls)

    def done(self, h) -> bool:
        h["polls"] -= 1
        return h["polls"] < 0

    def finish(self, h):
        self.busy -= 1
        return h["outs"]
