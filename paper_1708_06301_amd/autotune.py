"""Autotuner for the path kernels' launch shapes.

Results never depend on the launch shape (lanes per scanline of the
full-range and ragged kernels, and which scanlines of a ragged frame run on
packed registers); only speed does.  tune() times a caller-supplied workload under
each candidate egosgm_tuning with HIP events, keeps the fastest and caches it
in a JSON file keyed by image size, disparity range and device name.
"""
from __future__ import annotations

import itertools
import json
import os
import time

import torch

from . import egosgm as eg

CACHE = os.environ.get("EGOSGM_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "egosgm_tuning.json"))

# schedules 4-8 (grouped scanlines, alone or beside row scanlines) take no ragged_group
CANDIDATES = ([dict(full_group=f, ragged_group=r, ragged_schedule=s)
               for f, r, s in itertools.product((16, 32, 64), (16, 32, 64), (0, 1, 2, 3))] +
              [dict(full_group=f, ragged_group=32, ragged_schedule=s)
               for f, s in itertools.product((16, 32, 64), (4, 5, 6, 7, 8))])


def _kernel_version():
    """ABI version and a hash of the kernel source: a tuning measured on
    other kernels is never reused."""
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "egosgm_kernels.hip")
    try:
        with open(src, "rb") as fh:
            digest = hashlib.sha256(fh.read()).hexdigest()[:16]
    except OSError:
        digest = "nosrc"
    return f"abi{eg.abi_version()}-{digest}"


def _key(w, h, max_disp, tag=""):
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{name}|{_kernel_version()}|{w}x{h}|D{max_disp}|{tag}"


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(cache):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def time_workload(run, reps=3):
    """Median milliseconds of run() (which enqueues work on the current stream)."""
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(run, w, h, max_disp, tag="", candidates=None, reps=3, use_cache=True, log=None,
         margin=0.03):
    """Picks the fastest tuning for run() (the library default when it is
    within `margin` of the fastest), applies it and returns (tuning dict,
    {candidate index: ms})."""
    key = _key(w, h, max_disp, tag)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["tuning"]
        eg.set_tuning(**{**eg.get_tuning(), **best})
        return best, cache[key].get("times", {})
    cands = candidates or CANDIDATES
    times = {}
    run()  # warm caches and code objects
    torch.cuda.synchronize()
    t0 = time.time()
    for i, c in enumerate(cands):
        eg.set_tuning(**{**eg.get_tuning(), **c})
        times[i] = time_workload(run, reps)
        if log:
            log(f"tune {c}: {times[i]:.3f} ms")
    best_i = min(times, key=times.get)
    # Hysteresis: the library default stays unless a candidate is clearly
    # faster, so near-equal candidates do not flip from run to run.
    dflt = {k: eg.DEFAULT_TUNING[k] for k in cands[0]}
    d_i = next((i for i, c in enumerate(cands) if c == dflt), None)
    if d_i is not None and times[d_i] <= times[best_i] * (1.0 + margin):
        best_i = d_i
    best = cands[best_i]
    eg.set_tuning(**{**eg.get_tuning(), **best})
    if log:
        log(f"tuned in {time.time() - t0:.1f}s: {best} ({times[best_i]:.3f} ms)")
    if use_cache:
        cache[key] = {"tuning": best, "times": {str(k): v for k, v in times.items()}}
        _store(cache)
    return best, times


# batched plans: lanes per scanline x persistent path grid
PLAN_CANDIDATES = [dict(batch_group=g, batch_persistent=p) for g in (16, 32, 64) for p in (0, 1)]


def tune_plan(make_plan, key_tag, reps=3, use_cache=True, log=None):
    """Lanes per scanline and the persistent path grid of a batched plan,
    both fixed when the plan is built: builds one plan per candidate
    (make_plan() under that tuning), times its graph launch and keeps the
    fastest, cached under key_tag (the caller names the batch's shapes).
    Returns (candidate, plan, {"<group>/<persistent>": ms}); the other plans
    are closed."""
    key = _key(0, 0, 0, "plan|" + key_tag)
    cache = _load() if use_cache else {}
    base = eg.get_tuning()
    if use_cache and key in cache:
        best = cache[key]["tuning"]
        eg.set_tuning(**best)
        plan = make_plan()
        eg.set_tuning(**base)
        return best, plan, cache[key].get("times", {})
    best, times = None, {}
    for c in PLAN_CANDIDATES:
        eg.set_tuning(**c)
        p = make_plan()
        p.run()
        torch.cuda.synchronize()
        name = f"{c['batch_group']}/{c['batch_persistent']}"
        times[name] = time_workload(p.run, reps)
        if log:
            log(f"plan {c}: {times[name]:.3f} ms")
        if best is None or times[name] < best[2]:
            if best is not None:
                best[1].close()
            best = (c, p, times[name])
        else:
            p.close()
    eg.set_tuning(**base)
    if use_cache:
        cache = _load()
        cache[key] = {"tuning": best[0], "times": times}
        _store(cache)
    return best[0], best[1], times
