"""Serving many camera streams with continuous batching.

Every stream runs the per-frame method of Sec. 2 on its own: frame k is
predicted from the stream's own D^{k-1}, P^{k-1} and ego-motion (Sec. 2.2),
matched inside the prediction's windows (Sec. 2.3; the first frame, and the
first frame after a reset, over the full range) and fused by the Kalman
update (Sec. 2.4).  So a stream has at most one frame in flight and its
frames complete in order; different streams share nothing but the GPU.

The Server schedules:
  * admission: a stream reserves its device bytes (resident state plus its
    share of every in-flight slot's batch) against an HBM budget when it is
    opened; streams that do not fit wait, first in first out, until a close
    frees memory; a stream that could never fit is refused;
  * continuous batching: at every tick the oldest queued frame of each open,
    idle stream goes into one group, launched at once when a launch slot is
    free; frames that arrive while groups run join the next group, and the
    groups of different slots overlap on the device;
  * completion: latency = completion time - arrival time; a frame done after
    its deadline is counted late (and stays in the latency percentiles);
  * failures: an executor error tied to one stream marks that stream failed
    and drops its queue; the other streams of the group are launched again.

Executors do the work.  GpuExecutor runs a group as per-stream prediction
kernels, one batched matching launch (egosgm plan, updated per group) and
per-stream Kalman updates, all on the slot's HIP stream.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from .pipeline import Calib, FrameConfig


class AdmissionError(RuntimeError):
    """The stream can never fit in the HBM budget."""


class StreamFailed(RuntimeError):
    """An executor error that belongs to one stream."""

    def __init__(self, sid: int, msg: str = ""):
        super().__init__(f"stream {sid}: {msg}")
        self.sid = sid


@dataclass
class StreamSpec:
    w: int
    h: int
    calib: Calib
    cfg: FrameConfig = field(default_factory=FrameConfig)


@dataclass
class Request:
    sid: int
    seq: int
    left: object
    right: object
    R: object
    t: object
    arrival: float
    deadline: float
    reset: bool = False


@dataclass
class Result:
    sid: int
    seq: int
    arrival: float
    done: float
    status: str                 # "ok" or "failed"
    late: bool = False
    full_range: bool = False
    d: object = None
    p: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Stream:
    spec: StreamSpec
    need: int
    state: str = "pending"      # pending, open, failed, closed
    queue: collections.deque = field(default_factory=collections.deque)
    busy: bool = False
    closing: bool = False
    next_seq: int = 0
    reset_next: bool = False


class Server:
    def __init__(self, executor, hbm_budget: int, max_inflight: int | None = None,
                 deadline: float | None = None, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_inflight = max_inflight or getattr(executor, "n_slots", 1)
        self.deadline = deadline
        self.clock = clock
        self.used = 0
        self._streams: dict[int, _Stream] = {}
        self._pending: collections.deque = collections.deque()
        self._inflight: list = []            # (handle, [Request])
        self._next_sid = 0
        self.results: list[Result] = []
        self.refused = 0

    # ------------------------------------------------------------ streams
    def open_stream(self, spec: StreamSpec) -> int:
        need = int(self.ex.reserve_bytes(spec))
        if need > self.budget:
            self.refused += 1
            raise AdmissionError(f"stream needs {need} B, budget is {self.budget} B")
        sid = self._next_sid
        self._next_sid += 1
        self._streams[sid] = _Stream(spec, need)
        self._pending.append(sid)
        self._admit()
        return sid

    def state(self, sid: int) -> str:
        return self._streams[sid].state

    def close_stream(self, sid: int):
        s = self._streams[sid]
        if s.state == "pending":
            self._pending.remove(sid)
            s.state = "closed"
        elif s.busy:
            s.closing = True
        else:
            self._release(sid)
        self._admit()

    def reset_stream(self, sid: int):
        """The stream's next launched frame is matched over the full range
        (its prediction is dropped)."""
        self._streams[sid].reset_next = True

    def submit(self, sid: int, left, right, R=None, t=None, arrival: float | None = None) -> int:
        s = self._streams[sid]
        if s.state in ("failed", "closed") or s.closing:
            raise RuntimeError(f"stream {sid} is {s.state if not s.closing else 'closing'}")
        arrival = self.clock() if arrival is None else arrival
        deadline = arrival + self.deadline if self.deadline is not None else float("inf")
        seq = s.next_seq
        s.next_seq += 1
        s.queue.append(Request(sid, seq, left, right, R, t, arrival, deadline))
        return seq

    # ------------------------------------------------------------ scheduling
    def tick(self) -> list[Result]:
        """One scheduler pass: completions, admissions, launches."""
        done = self._complete()
        self._admit()
        self._launch()
        return done

    def idle(self) -> bool:
        return not self._inflight and not any(
            s.queue for s in self._streams.values() if s.state == "open")

    def drain(self, timeout: float = 60.0, poll: float = 0.0) -> list[Result]:
        out, t_end = [], self.clock() + timeout
        while not self.idle():
            out += self.tick()
            if self.clock() > t_end:
                raise TimeoutError("server did not drain")
            if poll:
                time.sleep(poll)
        return out

    def _admit(self):
        while self._pending:
            sid = self._pending[0]
            s = self._streams[sid]
            if self.used + s.need > self.budget:
                break
            self._pending.popleft()
            self.ex.open(sid, s.spec)
            self.used += s.need
            s.state = "open"

    def _release(self, sid: int):
        s = self._streams[sid]
        if s.state == "open":
            self.ex.close(sid)
            self.used -= s.need
        s.state = "closed"
        s.queue.clear()

    def _fail(self, sid: int, now: float) -> list[Result]:
        s = self._streams[sid]
        res = [Result(r.sid, r.seq, r.arrival, now, "failed") for r in s.queue]
        s.queue.clear()
        if s.state == "open":
            self.ex.close(sid)
            self.used -= s.need
        s.state = "failed"
        s.busy = False
        return res

    def _launch(self):
        while len(self._inflight) < self.max_inflight:
            group = []
            for sid, s in self._streams.items():
                if s.state == "open" and not s.busy and not s.closing and s.queue:
                    r = s.queue[0]
                    r.reset = s.reset_next
                    group.append(r)
            if not group:
                return
            try:
                handle = self.ex.launch(group)
            except StreamFailed as e:
                self.results += self._fail(e.sid, self.clock())
                continue
            for r in group:
                s = self._streams[r.sid]
                s.queue.popleft()
                s.busy = True
                if r.reset:
                    s.reset_next = False
            self._inflight.append((handle, group))

    def _complete(self) -> list[Result]:
        done, keep = [], []
        for handle, group in self._inflight:
            if not self.ex.done(handle):
                keep.append((handle, group))
                continue
            now = self.clock()
            outs = self.ex.finish(handle)
            for r, o in zip(group, outs):
                s = self._streams[r.sid]
                s.busy = False
                res = Result(r.sid, r.seq, r.arrival, now, "ok", late=now > r.deadline,
                             full_range=bool(o.get("full_range")), d=o.get("d"), p=o.get("p"))
                done.append(res)
                if s.closing:
                    s.closing = False
                    self._release(r.sid)
        self._inflight = keep
        self.results += done
        return done

    # ------------------------------------------------------------ statistics
    def stats(self) -> dict:
        ok = [r for r in self.results if r.status == "ok"]
        lat = np.array([r.latency for r in ok]) * 1e3
        span = (max(r.done for r in ok) - min(r.arrival for r in ok)) if ok else 0.0
        return {
            "frames": len(ok),
            "failed_frames": sum(r.status == "failed" for r in self.results),
            "late_frames": sum(r.late for r in ok),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3) if ok else None,
                           "p99": round(float(np.percentile(lat, 99)), 3) if ok else None,
                           "max": round(float(lat.max()), 3) if ok else None},
            "fps": round(len(ok) / span, 1) if span > 0 else None,
            "streams": {"open": sum(s.state == "open" for s in self._streams.values()),
                        "pending": len(self._pending),
                        "failed": sum(s.state == "failed" for s in self._streams.values()),
                        "refused": self.refused},
            "hbm_reserved_bytes": self.used,
        }


# ---------------------------------------------------------------- GPU executor
class GpuExecutor:
    """Runs groups on the GPU through the C ABI: per stream warp, refine and
    windows (or the full range), one batched matching launch of an egosgm
    plan over every open stream (the group's pairs active, the others
    skipped), per stream the Kalman update.  n_slots launch slots, each
    with its own HIP stream (default priority) and plan, so groups overlap.
    keep_outputs: results carry copies of the updated D^k, P^k."""

    def __init__(self, device="cuda", n_slots: int = 2, params=None, keep_outputs: bool = False):
        import torch
        from . import egosgm as eg
        self.torch, self.eg = torch, eg
        self.device = torch.device(device)
        self.n_slots = n_slots
        self.params = params
        self.keep = keep_outputs
        self.streams: dict = {}
        self.version = 0
        self.slots = [dict(stream=torch.cuda.Stream(self.device), plan=None, version=-1,
                           index={}, active=set(), busy=False, event=None, group=None)
                      for _ in range(n_slots)]

    # bytes -------------------------------------------------------------
    def reserve_bytes(self, spec: StreamSpec) -> int:
        n = spec.w * spec.h
        resident = n * (4 * 8 + 8 + 2 * 2 + 4 + 2) + 4
        resident += self.eg.lib().egosgm_windows_workspace_bytes(spec.w, spec.h)
        resident += self.eg.lib().egosgm_refine_workspace_bytes(spec.w, spec.h)
        per_slot = self.eg.lib().egosgm_sgm_workspace_bytes(spec.w, spec.h, spec.cfg.max_disp)
        per_slot += n * (2 + 4 + 4 + 2)                     # matcher outputs
        return resident + self.n_slots * per_slot

    # streams -----------------------------------------------------------
    def open(self, sid: int, spec: StreamSpec):
        from .pipeline import StreamState
        c = spec.cfg
        for e in self.streams.values():      # one plan: shared penalties and check
            o = e["spec"].cfg
            if (o.p1, o.p2, o.s_max, o.lr_tol) != (c.p1, c.p2, c.s_max, c.lr_tol):
                raise ValueError("streams of one executor share P1, P2, s_max and lr_tol")
        st = StreamState(spec.w, spec.h, spec.calib, spec.cfg, self.device, own_matcher=False)
        u8 = dict(dtype=self.torch.uint8, device=self.device)
        self.streams[sid] = dict(state=st, spec=spec,
                                 ph=(self.torch.zeros((spec.h, spec.w), **u8),
                                     self.torch.zeros((spec.h, spec.w), **u8)))
        self.version += 1

    def close(self, sid: int):
        self.streams.pop(sid, None)
        self.version += 1

    def _rebuild(self, slot):
        eg, torch = self.eg, self.torch
        if slot["plan"] is not None:
            slot["plan"].close()
        sids = sorted(self.streams)
        pairs = []
        for sid in sids:
            e = self.streams[sid]
            st, spec = e["state"], e["spec"]
            out = dict(disp_wta=torch.empty((spec.h, spec.w), dtype=torch.int16, device=self.device),
                       disp_sub=torch.empty((spec.h, spec.w), dtype=torch.float32, device=self.device),
                       var_meas=torch.empty((spec.h, spec.w), dtype=torch.float32, device=self.device),
                       disp_right=torch.empty((spec.h, spec.w), dtype=torch.int16, device=self.device))
            pairs.append(dict(left=e["ph"][0], right=e["ph"][1], max_disp=spec.cfg.max_disp,
                              windows=(st.lo, st.hi, st.off), out=out))
        c0 = self.streams[sids[0]]["spec"].cfg if sids else None
        prm = self.params or (eg.MatchParams(max(self.streams[s]["spec"].cfg.max_disp for s in sids),
                                             c0.p1, c0.p2, c0.s_max, c0.lr_tol) if sids else None)
        slot["plan"] = eg.Plan(pairs, prm, device=self.device) if pairs else None
        slot["index"] = {sid: i for i, sid in enumerate(sids)}
        slot["active"] = set(sids)      # every pair starts active: switched off at the first launch
        slot["version"] = self.version

    def reset(self, sid: int):
        self.streams[sid]["state"].reset()

    # groups ------------------------------------------------------------
    def launch(self, group):
        torch = self.torch
        slot = next(s for s in self.slots if not s["busy"])
        if slot["version"] != self.version:
            slot["stream"].synchronize()
            self._rebuild(slot)
        plan = slot["plan"]
        full = []
        # the frames may still be in flight on the caller's stream (an
        # asynchronous copy or rendering): the slot's work starts after it,
        # and the allocator keeps their memory until the slot is done
        slot["stream"].wait_stream(torch.cuda.current_stream(self.device))
        for r in group:
            for t in (r.left, r.right):
                if isinstance(t, torch.Tensor) and t.is_cuda:
                    t.record_stream(slot["stream"])
        with torch.cuda.stream(slot["stream"]):
            changes = []
            for r in group:
                st = self.streams[r.sid]["state"]
                if r.reset:
                    st.reset()
                full.append(st.full_range_next())
                win = st.predict(r.R, r.t)
                changes.append(dict(index=slot["index"][r.sid], active=True, left=r.left,
                                    right=r.right, windows=win))
            now_active = {r.sid for r in group}
            for sid in slot["active"] - now_active:
                if sid in slot["index"]:
                    changes.append(dict(index=slot["index"][sid], active=False))
            plan.update(changes)
            plan.run()
            outs = []
            for r, f in zip(group, full):
                st = self.streams[r.sid]["state"]
                st.filter(r.left, r.right, plan.outputs[slot["index"][r.sid]])
                d, p = st.update(out=plan.outputs[slot["index"][r.sid]])
                o = dict(full_range=f)
                if self.keep:
                    o["d"], o["p"] = d.clone(), p.clone()
                outs.append(o)
            ev = torch.cuda.Event()
            ev.record(slot["stream"])
        slot.update(busy=True, event=ev, group=group, outs=outs, active=now_active)
        return slot

    def done(self, slot) -> bool:
        return slot["event"].query()

    def finish(self, slot):
        slot["event"].synchronize()
        outs = slot["outs"]
        slot.update(busy=False, group=None, outs=None)
        return outs
