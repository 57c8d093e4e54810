"""Benchmark: ego-motion reduced census + SGM on one MI355X.

Headline workload: a 30-frame synthetic street sequence at 2048x1024 (ground
plane + 12 boxes + backdrop, f = 718*2048/1242 px, b = 0.54 m, 1 m/frame
forward with yaw ~ N(0, 0.5 deg)).  One step = one pass of the whole path
over the sequence: frame 0 is matched over the full range (D = 256); frames
1..29 warp the previous map by the ego-motion, refine the prediction, derive
windows of radius 6 around it, match only inside them and update the map
with the Kalman filter.  Census 9x7, 8 paths, P1 = 10, P2 = 120.  All stereo
pairs are resident in HBM before timing.

value = pixel*disparity*path updates per second (GCUPS) over the timed
steps.  Also reported: frames/s, per-frame latency p50/p99, the same
sequence with plain full-range SGM on every frame, the roofline of the
dominant kernel (HIP events around each stage on the library's stream,
over the timed region) and the CPU oracle timed on a bounded sample of the
same workload.  Further sections: the 20-frame 1242x375 sequence (D = 128,
r = 4) with its quality and variants, a batch of 32 mixed pairs in one
graph launch, and 16 served camera streams.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SGM GCUPS (pixel·disp·path/s) + frames/s, reduced vs full range; p99 latency"
HBM_PEAK_GBS = 8000.0

# The two sequence workloads: (name, w, h, frames, D, r, seed config index)
HIGHRES = ("highres", 2048, 1024, 30, 256, 6, 3)
STREET = ("street", 1242, 375, 20, 128, 4, 1)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_name(kind, w, h, D):
    tag = "highres" if (w, h) == (2048, 1024) else "street"
    return os.path.join(ROOT, "profiles", f"{kind}_{tag}_{w}x{h}_D{D}.json")


def _profile_entry(kind, w, h, D, kernel_name):
    """Per-dispatch counters of kernel_name from a committed rocprofv3
    summary, or None when there is none for this workload or the kernel
    source has changed since the counters were taken."""
    import hashlib
    try:
        prof = json.load(open(profile_name(kind, w, h, D)))
        src = open(os.path.join(ROOT, "paper_1708_06301_amd", "csrc", "egosgm_kernels.hip"), "rb").read()
    except (OSError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != prof.get("kernel_source_sha256"):
        return None
    return prof.get("kernels", {}).get(kernel_name)


def measured_traffic(w, h, D, kernel_name):
    """HBM bytes per dispatch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    k = _profile_entry("hbm_traffic", w, h, D, kernel_name)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def measured_valu_active(w, h, D, kernel_name):
    """SQ_ACTIVE_INST_VALU per dispatch (quad-cycles in which a SIMD's vector
    ALU issues, summed over all SIMDs)."""
    k = _profile_entry("sq_counters", w, h, D, kernel_name)
    return None if k is None else k.get("SQ_ACTIVE_INST_VALU")


def kernel_symbol(stage, tuning, D):
    """rocprofv3 name of the kernel a reduced frame launches for `stage`."""
    if stage == "paths":
        if tuning["ragged_schedule"] in (4, 5, 6, 7, 8):
            g = 16 if tuning["ragged_schedule"] in (5, 6) else 8
            dm = 64 if D <= 64 else (128 if D <= 128 else 256)
            if tuning["ragged_schedule"] == 8:
                return f"sgm_paths_regroup_kernel<{dm}, {6 if dm == 256 else 4}>"
            if tuning["ragged_schedule"] >= 6:
                return f"sgm_paths_hybrid_kernel<{g}, {dm}, 4, {1 if D <= 128 else 2}>"
            return f"sgm_paths_group_kernel<{g}, {dm}, 4>"
        if tuning["ragged_schedule"] == 3:
            return f"sgm_paths_reg_kernel<{1 if D <= 64 else (2 if D <= 128 else 4)}, 4>"
        g = tuning["ragged_group"]
        dr = 64 if D <= 64 else (128 if D <= 128 else 256)
        return (f"sgm_paths_ragged_kernel<{tuning['ragged_schedule']}, {1 if D <= 128 else 2}, {g}, "
                f"{dr // g}, 4>")
    if stage == "select":
        if tuning["ragged_schedule"] in (4, 5, 6, 7, 8):
            return "select_quad_kernel<8>"
        k = 1 if D <= 16 else (4 if D <= 64 else (8 if D <= 128 else 16))
        return f"sgm_select_kernel<16, {k}, 0, 8>"
    return None


# ---------------------------------------------------------------- sequences
def build_sequence(n_frames, w, h, seed_cfg, device):
    import torch
    from paper_1708_06301_amd import pipeline, synth
    seq = synth.street_sequence(w, h, n_frames, seed=synth.seed_for(seed_cfg))
    frames, gts = [], []
    t0 = time.time()
    for k in range(n_frames):
        left, right, gt = seq.frame(k, device=device)
        frames.append((torch.from_numpy(left).to(device), torch.from_numpy(right).to(device)))
        gts.append(gt)
    log(f"rendered {n_frames} frames {w}x{h} in {time.time() - t0:.1f}s")
    return seq, frames, pipeline.motions(seq), gts


def run_sequence(state, frames, motions, events=None, stage_timing=False):
    """One step.  With stage_timing, the library's per-stage events are on
    for frames 1.. only, so the stage figures describe the reduced frames."""
    from paper_1708_06301_amd import egosgm as eg
    state.reset()
    for k, (L, R) in enumerate(frames):
        if stage_timing:
            eg.timing_enable(k > 0)
        if events is not None:
            events[k][0].record()
        if k == 0:
            state.step(L, R)
        else:
            state.step(L, R, *motions[k])
        if events is not None:
            events[k][1].record()
    if stage_timing:
        eg.timing_enable(False)


def searched_updates(state, frames, motions):
    """Sum over frames of 8 * searched disparities (synchronising pass)."""
    import torch
    state.reset()
    tot, per = 0, []
    n = state.w * state.h
    for k, (L, R) in enumerate(frames):
        if k == 0 or state.cfg.full_range_only:
            state.step(L, R) if k == 0 else state.step(L, R, *motions[k])
            s = n * state.cfg.max_disp
        else:
            state.step(L, R, *motions[k])
            torch.cuda.synchronize()
            s = state.searched_slots()
        per.append(s)
        tot += 8 * s
    return tot, per


def timed_steps(state, frames, motions, steps, with_events=True, stage_timing=False):
    import torch
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in frames] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        run_sequence(state, frames, motions, ev[s] if with_events else None, stage_timing)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat = np.array([[a.elapsed_time(b) for a, b in row] for row in ev]) if with_events else None
    return dt, lat


def frame_config(D, r):
    from paper_1708_06301_amd import pipeline
    return pipeline.FrameConfig(max_disp=D, p1=10, p2=120, s_max=80, lr_tol=1, q=0.5,
                                r_fixed=r, r_min=0, r_max=256, edge_tol=2.0, fill_tol=1.0)


def roofline(stages, per_frame, n, tuning, w, h, D):
    """Roofline of the dominant stage of the reduced frames.  Algorithmic
    bytes are what the method must move per launch:
      paths:  4 B per searched slot (the forward and backward sweeps of the
              aggregation exchange one uint16 partial sum, written and read)
              plus 50 B per pixel (census codes for both sweeps, window,
              outputs), i.e. (4|W| + 50) / (8|W|) B per path update;
      select: the aggregated sum read once (2 B per slot) plus 12 B per
              pixel (window, outputs, right-map key).
    achieved = those bytes / the stage's average launch time (library
    events on the kernel's stream over the timed region)."""
    dom = max(stages, key=lambda s: stages[s][0])
    dom_ms, dom_n = stages[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    S_red = float(np.mean(per_frame[1:]))
    if dom == "paths":
        alg = 4 * S_red + 50 * n
    elif dom == "select":
        alg = 2 * S_red + 12 * n
    else:
        return None
    kname = kernel_symbol(dom, tuning, D)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(w, h, D, kname) if kname else None
    act = measured_valu_active(w, h, D, kname) if kname else None
    return dict(kernel=dom, symbol=kname, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                traffic_over_alg=None if traffic is None else round(traffic / alg, 3),
                avg_launch_ms=round(avg_ms, 4), launches=dom_n, alg_bytes_per_launch=int(alg),
                # what does bound the kernel: the fraction of SIMD cycles in
                # which the vector ALU issues (256 CUs at the 2.4 GHz peak clock)
                valu_busy=None if act is None else round(act / (256 * avg_ms * 1e-3 * 2.4e9), 3))


def measure_sequence(spec, args, dev, tune=True):
    """Times one sequence workload: the reduced pipeline, the same frames
    with full-range SGM on every frame, frame latencies, per-stage times
    and the dominant kernel's roofline."""
    import torch
    from paper_1708_06301_amd import autotune, pipeline
    from paper_1708_06301_amd import egosgm as eg
    name, w, h, nf, D, r, seed_cfg = spec
    seq, frames, motions, gts = build_sequence(nf, w, h, seed_cfg, dev)
    calib = pipeline.camera_of(seq)
    cfg = frame_config(D, r)
    red = pipeline.StreamState(w, h, calib, cfg, dev)
    cfg_full = pipeline.FrameConfig(**{**cfg.__dict__, "full_range_only": True})
    full = pipeline.StreamState(w, h, calib, cfg_full, dev)
    if tune:
        tuning, _ = autotune.tune(lambda: run_sequence(red, frames, motions), w, h, D, tag=name,
                                  use_cache=not args.retune, log=log)
    else:
        tuning = eg.get_tuning()
    tuning = {k: tuning[k] for k in ("full_group", "ragged_group", "ragged_schedule")}
    eg.set_tuning(**tuning)
    upd_red, per_frame = searched_updates(red, frames, motions)
    upd_full, _ = searched_updates(full, frames, motions)
    n = w * h
    search_frac = [s / (n * D) for s in per_frame]

    # a cached tuning skips the tuner's passes: keep the GPU busy for about a
    # second first, so that the timed steps never start from idle clocks
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < 1.0:
        run_sequence(red, frames, motions)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        run_sequence(red, frames, motions)
        run_sequence(full, frames, motions)
    torch.cuda.synchronize()

    # the timed region: exactly `steps` steps of the reduced pipeline with no
    # instrumentation (the throughput figures), then the same for the full
    # range; frame latencies come from a second pass with one event pair per
    # frame, and the per-stage figures from a third pass with the library's
    # stage events on (both add launch overhead of their own)
    dt, _ = timed_steps(red, frames, motions, args.steps, with_events=False)
    dt_full, _ = timed_steps(full, frames, motions, args.steps, with_events=False)
    _, lat = timed_steps(red, frames, motions, args.steps)
    _, lat_full = timed_steps(full, frames, motions, args.steps)
    eg.timing_read()
    timed_steps(red, frames, motions, args.steps, with_events=False, stage_timing=True)
    stages = eg.timing_read()
    stages = {k: v for k, v in stages.items() if v[1]}

    red_lat = lat[:, 1:].ravel()
    fps, fps_full = nf * args.steps / dt, nf * args.steps / dt_full
    out = {
        "gcups": round(upd_red * args.steps / dt / 1e9, 2),
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "workload": f"street sequence {w}x{h}, {nf} frames: frame 0 full SGM D={D}, frames 1-{nf - 1} "
                    f"warp + refine + Kalman (f32) + reduced SGM r=+-{r}; census 9x7, 8 paths, "
                    "P1=10, P2=120",
        "w": w, "h": h, "frames": nf, "max_disp": D, "r": r,
        "fps": round(fps, 1),
        "frame_latency_ms": {"p50": round(float(np.percentile(red_lat, 50)), 4),
                             "p99": round(float(np.percentile(red_lat, 99)), 4),
                             "frame0": round(float(np.median(lat[:, 0])), 4)},
        "full_range": {"gcups": round(upd_full * args.steps / dt_full / 1e9, 2), "fps": round(fps_full, 1),
                       "ms_per_step": round(dt_full / args.steps * 1e3, 3),
                       "frame_latency_ms_p50": round(float(np.percentile(lat_full.ravel(), 50)), 4)},
        "speedup_vs_full": round(fps / fps_full, 3),
        "search_fraction": {"mean_reduced": round(float(np.mean(search_frac[1:])), 4),
                            "per_frame": [round(x, 4) for x in search_frac]},
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "roofline": roofline(stages, per_frame, n, tuning, w, h, D),
        "tuning": tuning,
    }
    ctx = dict(seq=seq, frames=frames, motions=motions, gts=gts, cfg=cfg, red=red, full=full,
               calib=calib)
    return out, ctx


# ---------------------------------------------------------------- CPU oracle
def _oracle_band_loop(left, right, motions, cam, cfg, y0, y1, n_frames, budget_s):
    """The oracle's own frame loop on rows y0..y1-1 of the sequence (a band
    matched as an image of its own; the principal point moves with it):
    frame 0 over the full range, then warp + refine + windows + reduced SGM
    + Kalman, until n_frames frames or budget_s seconds.  Returns (path
    updates, seconds, frames done)."""
    from oracle import oracle as orc
    f, cx, cy, b = cam
    cy = cy - y0
    t0 = time.perf_counter()
    upd, d, p, k = 0, None, None, 0
    while k < n_frames:
        L = np.ascontiguousarray(left[k, y0:y1])
        R = np.ascontiguousarray(right[k, y0:y1])
        if k == 0:
            o = orc.sgm(L, R, cfg["D"], cfg["p1"], cfg["p2"], cfg["s_max"], cfg["lr_tol"])
            upd += 8 * L.size * cfg["D"]
            dk, pk = orc.kalman(np.full(L.shape, -1, np.float32), np.zeros(L.shape, np.float32),
                                o["disp_sub"].astype(np.float32), o["var_meas"].astype(np.float32))
        else:
            Rm, t = motions[k, :9].reshape(3, 3), motions[k, 9:]
            wp = orc.warp(d, p, Rm, t, f, cx, cy, b, cfg["q"])
            dp, pp = orc.refine(wp["d_pred"].astype(np.float32), wp["p_pred"].astype(np.float32),
                                cfg["edge_tol"], cfg["fill_tol"])
            win = orc.windows(dp, pp, cfg["D"], r_fixed=cfg["r"], r_min=0, r_max=256)
            o = orc.sgm(L, R, cfg["D"], cfg["p1"], cfg["p2"], cfg["s_max"], cfg["lr_tol"], windows=win)
            upd += 8 * int(win[2][-1])
            dk, pk = orc.kalman(dp, pp, o["disp_sub"].astype(np.float32),
                                o["var_meas"].astype(np.float32))
        d, p = dk.astype(np.float32), pk.astype(np.float32)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return upd, time.perf_counter() - t0, k


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_worker():
    """One oracle instance of the parallel CPU figure, in a child process
    started before the parent touched the GPU: it waits for one job line
    (JSON: dir, y0, y1, frames, budget, out) on stdin, runs it and exits;
    an empty line or end of input means no job."""
    line = sys.stdin.readline().strip()
    if not line:
        return 0
    job = json.loads(line)
    d = job["dir"]
    left = np.load(os.path.join(d, "left.npy"), mmap_mode="r")
    right = np.load(os.path.join(d, "right.npy"), mmap_mode="r")
    motions = np.load(os.path.join(d, "motions.npy"))
    meta = json.load(open(os.path.join(d, "meta.json")))
    upd, sec, k = _oracle_band_loop(left, right, motions, meta["cam"], meta["cfg"], job["y0"], job["y1"],
                                    job["frames"], job["budget"])
    json.dump(dict(upd=upd, sec=sec, frames=k), open(job["out"], "w"))
    return 0


class CpuPool:
    """Child processes for the parallel CPU figure, one per core (at most
    16, the CPU share of one GPU on the box).  They are started before this
    process initialises the GPU, so no child inherits a GPU context, and
    they idle on stdin until run() hands each its job."""

    def __init__(self):
        self.n = max(1, min(16, len(os.sched_getaffinity(0))))
        self.procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker"],
                                       stdin=subprocess.PIPE, text=True) for _ in range(self.n)]

    def run(self, jobs):
        for p, j in zip(self.procs, jobs):
            p.stdin.write(json.dumps(j) + "\n")
            p.stdin.flush()
        return self.close()

    def close(self):
        ok = True
        for p in self.procs:
            try:
                p.stdin.close()
            except OSError:
                pass
            ok = p.wait() == 0 and ok
        self.procs = []
        return ok


def cpu_baseline(seq, frames, motions, cfg, pool=None, budget_s=20.0, band=128, par_frames=6):
    """The plain single-threaded C oracle on bounded samples of the headline
    workload.  (i) One instance on one core: the oracle's frame loop over a
    band of `band` rows through the middle of the same frames (frame 0 full
    range, then reduced frames) until about budget_s seconds.  (ii) With a
    CpuPool, one instance per pool process and core, each on its own band of
    rows so the bands tile the whole image, over the first par_frames
    frames, all at once; its figure is the total updates over the wall
    time."""
    from oracle import oracle as orc
    orc.build(force=False)
    nf = len(frames)
    w, h = seq.cam.w, seq.cam.h
    left = np.stack([np.asarray(L) for L, _ in frames])
    right = np.stack([np.asarray(R) for _, R in frames])
    mot = np.zeros((nf, 12))
    for k in range(1, nf):
        Rm, t = motions[k]
        mot[k, :9] = np.asarray(Rm).ravel()
        mot[k, 9:] = np.asarray(t).ravel()
    cam = [seq.cam.f, seq.cam.cx, seq.cam.cy, seq.cam.baseline]
    c = dict(D=cfg.max_disp, p1=cfg.p1, p2=cfg.p2, s_max=cfg.s_max, lr_tol=cfg.lr_tol, q=cfg.q,
             edge_tol=cfg.edge_tol, fill_tol=cfg.fill_tol, r=cfg.r_fixed)
    y0 = max(0, h // 2 - band // 2)
    y1 = min(h, y0 + band)
    upd1, sec1, k1 = _oracle_band_loop(left, right, mot, cam, c, y0, y1, nf, budget_s)
    par = None
    if pool is not None:
        n_work = pool.n
        with tempfile.TemporaryDirectory(prefix="egosgm_cpu_") as tmp:
            np.save(os.path.join(tmp, "left.npy"), left[:par_frames])
            np.save(os.path.join(tmp, "right.npy"), right[:par_frames])
            np.save(os.path.join(tmp, "motions.npy"), mot[:par_frames])
            json.dump(dict(cam=cam, cfg=c), open(os.path.join(tmp, "meta.json"), "w"))
            cuts = [round(i * h / n_work) for i in range(n_work + 1)]
            jobs = [dict(dir=tmp, y0=cuts[i], y1=cuts[i + 1], frames=par_frames, budget=4 * budget_s,
                         out=os.path.join(tmp, f"out{i}.json")) for i in range(n_work)]
            t0 = time.perf_counter()
            ok = pool.run(jobs)
            wall = time.perf_counter() - t0
            if ok:
                res = [json.load(open(j["out"])) for j in jobs]
                par = dict(value=round(sum(r["upd"] for r in res) / wall / 1e9, 4), unit="GCUPS",
                           cores=n_work, wall_s=round(wall, 1),
                           sample=f"frames 0..{min(r['frames'] for r in res) - 1} of the same sequence, "
                                  f"the image cut into {n_work} row bands of about {h // n_work} rows "
                                  "(each matched on its own), one single-threaded oracle instance per "
                                  "band and core, all at once")
    return dict(value=round(upd1 / sec1 / 1e9, 4), unit="GCUPS", cores=1, kind="oracle",
                cpu_model=_cpu_model(),
                sample=f"rows {y0}..{y1 - 1} (a {w}x{y1 - y0} band matched on its own) of frames "
                       f"0..{k1 - 1} of the same sequence: frame 0 full range D={cfg.max_disp}, then "
                       f"warp + refine + windows r={cfg.r_fixed} + reduced SGM + Kalman; "
                       f"single-threaded plain C oracle, {sec1:.1f} s",
                all_cores=par)


# ---------------------------------------------------------------- sections
def batch_section(dev, n_pairs, steps, log):
    """32 mixed stereo pairs (640x192 D=64, 960x288 D=96, 1242x375 D=128) with
    per-pixel windows r = clamp(ceil(3 sqrt(p)), 2, 16) taken from each pair's
    own frame-1 prediction; the reduced matching of all pairs is one plan
    (one graph launch).  Compared with the same batch over the full range and
    with 32 single-pair calls."""
    import torch
    from paper_1708_06301_amd import egosgm as eg
    from paper_1708_06301_amd import pipeline, synth
    sizes = [(640, 192, 64), (960, 288, 96), (1242, 375, 128)]
    states, cases, full_cases = [], [], []
    t0 = time.time()
    for i in range(n_pairs):
        w, h, D = sizes[i % 3]
        seq = synth.street_sequence(w, h, 2, seed=synth.seed_for(2, i))
        (L0, R0, _), (L1, R1, _) = seq.frame(0, device=dev), seq.frame(1, device=dev)
        L0, R0, L1, R1 = (torch.from_numpy(a).to(dev) for a in (L0, R0, L1, R1))
        cfg = pipeline.FrameConfig(max_disp=D, r_fixed=-1, r_min=2, r_max=16)
        st = pipeline.StreamState(w, h, pipeline.camera_of(seq), cfg, dev)
        st.step(L0, R0)
        win = st.predict(*[np.asarray(a, np.float64) for a in seq.motion(1)])
        states.append(st)
        cases.append(dict(left=L1, right=R1, max_disp=D, windows=win))
        full_cases.append(dict(left=L1, right=R1, max_disp=D))
    torch.cuda.synchronize()
    log(f"batch: {n_pairs} pairs prepared in {time.time() - t0:.1f}s")
    slots = sum(int(st.off[st.w * st.h].item()) & 0xFFFFFFFF for st in states)
    full_slots = sum(st.w * st.h * st.cfg.max_disp for st in states)
    pixels = sum(st.w * st.h for st in states)
    prm = eg.MatchParams()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, bb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        bb.record()
        bb.synchronize()
        return a.elapsed_time(bb) / reps

    reps = max(3, steps)
    # Lanes per scanline are fixed when a plan is built: the autotuner builds
    # one plan per candidate and keeps the fastest (cached per batch shape),
    # for the reduced and the full batch.
    from paper_1708_06301_amd import autotune
    shape = "+".join(f"{w}x{h}D{D}" for w, h, D in sizes) + f"x{n_pairs}"
    best_g, plan, group_ms = autotune.tune_plan(lambda: eg.Plan(cases, prm), "ragged|" + shape, reps=reps, log=log)
    best_gf, plan_full, group_ms_full = autotune.tune_plan(lambda: eg.Plan(full_cases, prm), "full|" + shape,
                                                           reps=reps, log=log)
    ms_red = timed(plan.run, reps)
    ms_full = timed(plan_full.run, reps)
    singles = [dict(left=c["left"], right=c["right"], win=c["windows"],
                    prm=eg.MatchParams(c["max_disp"]), out=st.out, ws=st.ws)
               for c, st in zip(cases, states)]

    def run_singles():
        for s in singles:
            eg.sgm_reduced(s["left"], s["right"], *s["win"], s["prm"], out=s["out"], workspace=s["ws"])

    ms_single = timed(run_singles, reps)
    eg.timing_read()
    eg.timing_enable(True)
    for _ in range(reps):
        plan.run(eager=True)
    eg.timing_enable(False)
    st_ms = eg.timing_read()
    torch.cuda.synchronize()
    paths_ms, paths_n = st_ms["batch_paths"]
    avg = paths_ms / max(paths_n, 1)
    alg = 4 * slots + 50 * pixels            # the aggregation's bytes (4|W| + 50 per pixel)
    achieved = alg / (avg * 1e-3) / 1e9
    out = {
        "workload": f"{n_pairs} pairs (640x192 D=64, 960x288 D=96, 1242x375 D=128), windows "
                    "r=clamp(ceil(3 sqrt(p)),2,16) from each pair's frame-1 prediction, one graph launch",
        "gcups": round(8 * slots / (ms_red * 1e-3) / 1e9, 1),
        "ms_per_batch": round(ms_red, 4),
        "plan_tuning": best_g,
        "ms_per_batch_by_plan_tuning": {k: round(v, 4) for k, v in group_ms.items()},
        "pairs_per_s": round(n_pairs / (ms_red * 1e-3), 1),
        "search_fraction": round(slots / full_slots, 4),
        "full_range": {"gcups": round(8 * full_slots / (ms_full * 1e-3) / 1e9, 1),
                       "ms_per_batch": round(ms_full, 4), "plan_tuning": best_gf,
                       "ms_per_batch_by_plan_tuning": {k: round(v, 4) for k, v in group_ms_full.items()}},
        "speedup_vs_full": round(ms_full / ms_red, 3),
        "single_pair_calls_ms": round(ms_single, 4),
        "speedup_vs_single_calls": round(ms_single / ms_red, 3),
        "stages_ms_eager": {k[6:]: round(v[0] / max(v[1], 1), 4) for k, v in st_ms.items()
                            if k.startswith("batch_") and v[1]},
        "roofline_paths": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "avg_launch_ms": round(avg, 4), "alg_bytes_per_launch": int(alg)},
    }
    plan.close()
    plan_full.close()
    return out


def quality_section(red, full, frames, motions, gts, max_disp):
    """Bad-pixel rates against the renderer's ground truth (Sec. 3's metric):
    plain full-range SGM on every frame, the reduced pipeline's own
    measurement, and its Kalman-filtered map D^k; frames 1.. (frame 0 is
    the same full-range match for all three)."""
    import torch
    from paper_1708_06301_amd.quality import bad_pixels, summarise
    out = {"full_sgm": [], "reduced_measurement": [], "reduced_filtered": []}
    red.reset()
    full.reset()
    for k, (L, R) in enumerate(frames):
        Rm, t = motions[k] if k > 0 else (None, None)
        d_red, _ = red.step(L, R, Rm, t)
        full.step(L, R, Rm, t)
        torch.cuda.synchronize()
        if k == 0:
            continue
        out["full_sgm"].append(bad_pixels(full.out["disp_sub"], gts[k], max_disp))
        out["reduced_measurement"].append(bad_pixels(red.out["disp_sub"], gts[k], max_disp))
        out["reduced_filtered"].append(bad_pixels(d_red, gts[k], max_disp))
    return {"frames": f"1..{len(frames) - 1}", "threshold": "3 px or/and 5% of the true disparity",
            **{k: summarise(v) for k, v in out.items()}}


def variants_section(w, h, calib, cfg, frames, motions, gts, dev, reps=3):
    """Variants on the same sequence: 4 paths (rows and columns only), the
    SAD check (radius 2, at most 600, i.e. a mean absolute difference of 24
    per pixel) after the left-right check, and the left-right check of the
    prediction (the warped right map, tolerance 1 px) before the windows.
    Time per step (median of reps, HIP events) and the filtered map's
    bad-pixel rates."""
    import torch
    from paper_1708_06301_amd import pipeline
    from paper_1708_06301_amd.quality import bad_pixels, summarise
    out = {}
    for name, kw in (("paths4", dict(n_paths=4)), ("sad_check", dict(sad_radius=2, sad_max=600)),
                     ("lr_predict", dict(lr_predict=True, lr_predict_tol=1.0)),
                     ("paths4_full_range", dict(n_paths=4, full_range_only=True))):
        st = pipeline.StreamState(w, h, calib, pipeline.FrameConfig(**{**cfg.__dict__, **kw}), dev)
        times = []
        for _ in range(reps + 1):
            a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            st.reset()
            a.record()
            for k, (L, R) in enumerate(frames):
                st.step(L, R, *(motions[k] if k > 0 else (None, None)))
            b_.record()
            b_.synchronize()
            times.append(a.elapsed_time(b_))
        ms = sorted(times[1:])[len(times[1:]) // 2]
        q = []
        st.reset()
        for k, (L, R) in enumerate(frames):
            d, _ = st.step(L, R, *(motions[k] if k > 0 else (None, None)))
            if k > 0:
                torch.cuda.synchronize()
                q.append(bad_pixels(d, gts[k], cfg.max_disp))
        out[name] = {"ms_per_step": round(ms, 3), "fps": round(len(frames) / (ms * 1e-3), 1),
                     "quality_filtered": summarise(q)}
    return out


def vo_section(w, h, calib, cfg, frames, motions, gts, dev, reps=3):
    """Ego-motion from the images (FrameConfig.vo, estimate_motion) in place
    of the renderer's exact motion on the same sequence: per-frame pose error
    against that motion, the search fraction and the filtered map's bad-pixel
    rates beside the exact-motion pipeline's, the estimate's own time per
    frame (library stage events) and the time per step (median of reps, HIP
    events; each frame reads its estimate back to the host for the warp)."""
    import torch
    from paper_1708_06301_amd import egosgm as eg, pipeline
    from paper_1708_06301_amd.quality import bad_pixels, summarise
    st = pipeline.StreamState(w, h, calib, pipeline.FrameConfig(**{**cfg.__dict__, "vo": True}), dev)
    gt_st = pipeline.StreamState(w, h, calib, cfg, dev)
    t_err, r_err, frac, frac_gt, q, q_gt = [], [], [], [], [], []
    st.reset()
    gt_st.reset()
    for k, (L, R) in enumerate(frames):
        d, _ = st.step(L, R)
        d_gt, _ = gt_st.step(L, R, *(motions[k] if k > 0 else (None, None)))
        torch.cuda.synchronize()
        if k == 0:
            continue
        Re, te = st.vo_motion
        Rg, tg = motions[k]
        dR = Re @ np.asarray(Rg).T
        t_err.append(float(np.linalg.norm(te - np.asarray(tg))))
        r_err.append(float(np.degrees(np.arccos(np.clip((np.trace(dR) - 1.0) / 2.0, -1.0, 1.0)))))
        frac.append(st.searched_slots() / (w * h * cfg.max_disp))
        frac_gt.append(gt_st.searched_slots() / (w * h * cfg.max_disp))
        q.append(bad_pixels(d, gts[k], cfg.max_disp))
        q_gt.append(bad_pixels(d_gt, gts[k], cfg.max_disp))
    times = []
    for _ in range(reps + 1):
        a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.reset()
        a.record()
        for L, R in frames:
            st.step(L, R)
        b_.record()
        b_.synchronize()
        times.append(a.elapsed_time(b_))
    ms = sorted(times[1:])[len(times[1:]) // 2]
    eg.timing_enable(True)
    eg.timing_read()
    st.reset()
    for L, R in frames:
        st.step(L, R)
    torch.cuda.synchronize()
    stg = eg.timing_read()
    eg.timing_enable(False)
    vo_ms = stg["vo"][0] / max(1, stg["vo"][1])
    return {"frames": f"1..{len(frames) - 1}", "levels": int(st.vo_prm.levels),
            "iters": list(st.vo_prm.iters[:st.vo_prm.levels]),
            "translation_error_m": {"mean": round(float(np.mean(t_err)), 5), "max": round(float(np.max(t_err)), 5)},
            "rotation_error_deg": {"mean": round(float(np.mean(r_err)), 5), "max": round(float(np.max(r_err)), 5)},
            "estimate_ms_per_frame": round(vo_ms, 4), "ms_per_step": round(ms, 3),
            "search_fraction": {"vo": round(float(np.mean(frac)), 4), "exact_motion": round(float(np.mean(frac_gt)), 4)},
            "quality_filtered": {"vo": summarise(q), "exact_motion": summarise(q_gt)}}


def serve_section(dev, n_frames, log, budget_gib=32.0):
    """16 camera streams (8 at 1242x375 D=128, 8 at 640x192 D=64), n_frames
    synthetic street frames each, arriving at 30 fps with Poisson jitter,
    served with continuous batching (2 launch slots) in real time: p50/p99
    frame latency (arrival to completion), fps, frames later than one frame
    period.  Then the same frames all queued at once (capacity), reduced and
    full range, for the served speedup over full-range SGM."""
    import torch
    from paper_1708_06301_amd import pipeline, synth
    from paper_1708_06301_amd.serve import GpuExecutor, Server, StreamSpec
    kinds = [(1242, 375, 128)] * 8 + [(640, 192, 64)] * 8
    streams = []
    t0 = time.time()
    for i, (w, h, D) in enumerate(kinds):
        seq = synth.street_sequence(w, h, n_frames, seed=synth.seed_for(5, i))
        frames = []
        for k0 in range(0, n_frames, 8):
            frames += synth.render_frames_device(seq.scene, seq.cam,
                                                 list(range(k0, min(n_frames, k0 + 8))), dev)
        streams.append(dict(seq=seq, frames=frames, motions=pipeline.motions(seq),
                            cfg=pipeline.FrameConfig(max_disp=D, r_fixed=4)))
        log(f"serve: stream {i} ({w}x{h}) {n_frames} frames rendered, {time.time() - t0:.1f}s")
    torch.cuda.synchronize()
    rate = 30.0
    g = np.random.default_rng(synth.seed_for(6))
    arrivals = []
    for i in range(len(streams)):
        t = g.uniform(0, 1 / rate) + np.cumsum(g.exponential(1 / rate, n_frames))
        arrivals += [(float(t[k]), i, k) for k in range(n_frames)]
    arrivals.sort()

    def run(full_only, realtime):
        ex = GpuExecutor(dev, n_slots=2)
        srv = Server(ex, hbm_budget=int(budget_gib * (1 << 30)), deadline=1.0 / rate)
        ids = []
        for s in streams:
            cfg = s["cfg"] if not full_only else pipeline.FrameConfig(
                **{**s["cfg"].__dict__, "full_range_only": True})
            ids.append(srv.open_stream(StreamSpec(s["frames"][0][0].shape[1],
                                                  s["frames"][0][0].shape[0],
                                                  pipeline.camera_of(s["seq"]), cfg)))
        # warm-up: one frame of every stream (plan build, code objects), then reset
        for i, s in enumerate(streams):
            srv.submit(ids[i], *s["frames"][0])
        srv.drain(timeout=120)
        for i in ids:
            srv.reset_stream(i)
        srv.results.clear()
        torch.cuda.synchronize()
        start = time.perf_counter()
        j = 0
        while j < len(arrivals) or not srv.idle():
            now = time.perf_counter() - start
            while j < len(arrivals) and (not realtime or arrivals[j][0] <= now):
                ta, i, k = arrivals[j]
                s = streams[i]
                R, t = s["motions"][k] if k > 0 else (None, None)
                srv.submit(ids[i], *s["frames"][k], R, t,
                           arrival=start + (ta if realtime else 0.0))
                j += 1
            srv.tick()
            if realtime and srv.idle() and j < len(arrivals):
                time.sleep(min(5e-4, max(0.0, arrivals[j][0] - (time.perf_counter() - start))))
        torch.cuda.synchronize()
        st = srv.stats()
        st["makespan_s"] = round(time.perf_counter() - start, 3)
        return st

    rt = run(False, True)
    log(f"serve: real time {rt}")
    cap = run(False, False)
    log(f"serve: capacity reduced {cap}")
    cap_full = run(True, False)
    log(f"serve: capacity full range {cap_full}")
    return {
        "workload": f"16 streams (8 at 1242x375 D=128, 8 at 640x192 D=64), {n_frames} frames each, "
                    "Poisson arrivals at 30 fps, windows r=4 from each stream's own prediction, "
                    "2 launch slots, deadline one frame period",
        "realtime": {k: rt[k] for k in ("frames", "fps", "latency_ms", "late_frames", "streams",
                                        "hbm_reserved_bytes", "makespan_s")},
        "capacity_fps": cap["fps"],
        "capacity_fps_full_range": cap_full["fps"],
        "speedup_vs_full": round(cap["fps"] / cap_full["fps"], 3) if cap_full["fps"] else None,
        "capacity_latency_ms": cap["latency_ms"],
    }


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--cpu-worker":
        return cpu_worker()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("highres", "street"), default="highres",
                    help="headline sequence (the other one is reported as a section)")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline sequence only (no other section)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default tuning")
    ap.add_argument("--no-street", action="store_true", help="skip the 1242x375 section")
    ap.add_argument("--no-batch", action="store_true", help="skip the 32-pair batched section")
    ap.add_argument("--batch-pairs", type=int, default=32)
    ap.add_argument("--no-serve", action="store_true", help="skip the 16-stream serving section")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the variants section (its 4-path runs share the path kernel's symbol)")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-vo", action="store_true", help="skip the ego-motion-from-images sections")
    ap.add_argument("--serve-frames", type=int, default=300)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the path has no "
              "collective; streams and pairs shard across GPUs with no exchange.",
              file=sys.stderr)
        return 2

    # the CPU baseline's worker processes start before anything touches the GPU
    pool = CpuPool() if not args.no_cpu_baseline and not args.copy_calibration else None
    try:
        return run(args, pool)
    finally:
        if pool is not None:
            pool.close()


def run(args, pool):
    import torch
    from paper_1708_06301_amd import egosgm as eg

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_dispatch": 256 << 20, "dispatches": 5}))
        return 0
    eg.lib()
    head_spec, other_spec = (HIGHRES, STREET) if args.workload == "highres" else (STREET, HIGHRES)
    head, hctx = measure_sequence(head_spec, args, dev, tune=not args.no_tune)
    log(f"headline {head_spec[0]}: {head['gcups']} GCUPS, {head['ms_per_step']} ms per step")

    out = {
        "metric": METRIC,
        "value": head["gcups"],
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": head["workload"], "w": head["w"], "h": head["h"],
                   "frames": head["frames"], "max_disp": head["max_disp"], "r": head["r"]},
        **{k: head[k] for k in ("fps", "frame_latency_ms", "full_range", "speedup_vs_full",
                                "search_fraction", "stages_ms_per_step", "roofline", "tuning")},
    }
    if not args.only_headline and not args.no_quality:
        out["quality"] = quality_section(hctx["red"], hctx["full"], hctx["frames"], hctx["motions"],
                                         hctx["gts"], head["max_disp"])
    if not args.only_headline and not args.no_vo:
        out["vo"] = vo_section(head["w"], head["h"], hctx["calib"], hctx["cfg"], hctx["frames"], hctx["motions"],
                               hctx["gts"], dev)
        log(f"vo: {out['vo']}")
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle gets host copies of the frames; the GPU state is released first
        seq, frames, motions, cfg = hctx["seq"], hctx["frames"], hctx["motions"], hctx["cfg"]
        cpu = (seq, [(L.cpu().numpy(), R.cpu().numpy()) for L, R in frames], motions, cfg)
    del hctx
    torch.cuda.empty_cache()
    if not args.only_headline and not args.no_street:
        sec, sctx = measure_sequence(other_spec, args, dev, tune=not args.no_tune)
        if not args.no_quality:
            sec["quality"] = quality_section(sctx["red"], sctx["full"], sctx["frames"], sctx["motions"],
                                             sctx["gts"], sec["max_disp"])
        if not args.no_vo:
            sec["vo"] = vo_section(sec["w"], sec["h"], sctx["calib"], sctx["cfg"], sctx["frames"], sctx["motions"],
                                   sctx["gts"], dev)
        if not args.no_variants:
            sec["variants"] = variants_section(sec["w"], sec["h"], sctx["calib"], sctx["cfg"],
                                               sctx["frames"], sctx["motions"], sctx["gts"], dev)
        out[f"{other_spec[0]}_{other_spec[1]}x{other_spec[2]}"] = sec
        del sctx
        torch.cuda.empty_cache()
    if not args.only_headline and not args.no_batch:
        out["batched"] = batch_section(dev, args.batch_pairs, args.steps, log)
    if not args.only_headline and not args.no_serve:
        out["serving"] = serve_section(dev, args.serve_frames, log)
    if cpu is not None:
        out["cpu_baseline"] = cpu_baseline(*cpu, pool=pool, budget_s=args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
