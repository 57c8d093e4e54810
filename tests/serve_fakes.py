"""A CPU executor for the serving scheduler, backed by the oracle (test
infrastructure: it runs the method of Sec. 2 per stream with the plain C
oracle, so the scheduler's admission, ordering and failure handling can be
tested without a GPU)."""
from __future__ import annotations

import numpy as np

import oracle_frames
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
            f = oracle_frames.frame(L, R, None if full else e["d"], None if full else e["p"],
                                    None if full else (r.R, r.t), c, cfg)
            dk, pk = f["d"], f["p"]
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
