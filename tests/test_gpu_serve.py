"""GPU serving: plan updates (active pairs, images, windows) and the served
results of a stream, which must be the same alone, in a mix of streams,
and through the plain per-frame pipeline (bit-exact: the kernels of one
pair never read another pair's data)."""
import numpy as np
import pytest
import torch

from paper_1708_06301_amd import egosgm as eg
from paper_1708_06301_amd import pipeline, synth
from paper_1708_06301_amd.serve import GpuExecutor, Server, StreamSpec

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print("CASE", *a, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _pair(w, h, seed, shift):
    left = synth.texture(w, h, seed, noise_sigma=8.0, scale=5.0)
    right = np.roll(left, -shift, axis=1)
    return _gpu(left), _gpu(right)


def _windows(w, h, D, seed, r=3):
    g = np.random.default_rng(seed)
    d = g.uniform(0, D - 1, (h, w)).astype(np.float32)
    d[g.random((h, w)) < 0.1] = -1.0
    return eg.windows_from_prediction(_gpu(d), None, D, r_fixed=r)


def _same(a, b):
    return all(torch.equal(a[k], b[k]) for k in ("disp_wta", "disp_sub", "var_meas", "disp_right"))


def test_plan_update_active_images_and_windows():
    _say("plan update: 3 pairs")
    shapes = [(70, 23, 64), (45, 30, 32), (96, 17, 128)]
    pairs = []
    for i, (w, h, D) in enumerate(shapes):
        L, R = _pair(w, h, 900 + i, 5 + i)
        pairs.append(dict(left=L, right=R, max_disp=D, windows=_windows(w, h, D, 950 + i)))
    plan = eg.Plan(pairs, eg.MatchParams())
    plan.run()
    for q, o in zip(pairs, plan.outputs):
        ref = eg.sgm_reduced(q["left"], q["right"], *q["windows"], eg.MatchParams(q["max_disp"]))
        torch.cuda.synchronize()
        assert _same(o, ref)
    # pair 1 off (its outputs must stay), pair 0 to the full range, pair 2 new images
    plan.outputs[1]["disp_wta"].fill_(-7)
    L2, R2 = _pair(96, 17, 990, 9)
    plan.update([dict(index=1, active=False), dict(index=0, windows=None),
                 dict(index=2, left=L2, right=R2)])
    plan.run()
    torch.cuda.synchronize()
    assert bool((plan.outputs[1]["disp_wta"] == -7).all())
    ref0 = eg.sgm_full(pairs[0]["left"], pairs[0]["right"], eg.MatchParams(64))
    ref2 = eg.sgm_reduced(L2, R2, *pairs[2]["windows"], eg.MatchParams(128))
    torch.cuda.synchronize()
    assert _same(plan.outputs[0], ref0) and _same(plan.outputs[2], ref2)
    # pair 1 back on with new windows
    win1 = _windows(45, 30, 32, 999, r=5)
    plan.update([dict(index=1, active=True, windows=win1)])
    plan.run()
    ref1 = eg.sgm_reduced(pairs[1]["left"], pairs[1]["right"], *win1, eg.MatchParams(32))
    torch.cuda.synchronize()
    assert _same(plan.outputs[1], ref1)
    with pytest.raises(eg.EgoSgmError):
        plan.update([dict(index=3, active=False)])
    plan.close()


def _sequence(w, h, n, seed):
    seq = synth.street_sequence(w, h, n, seed=synth.seed_for(7, seed))
    frames = []
    for k in range(n):
        L, R, _ = seq.frame(k, device=DEV)
        frames.append((torch.from_numpy(L).to(DEV), torch.from_numpy(R).to(DEV)))
    return seq, frames, pipeline.motions(seq)


def _serve(streams, order, slots=2):
    """streams: list of (seq, frames, motions, cfg); order: (stream, k) in
    arrival order.  Returns per stream the list of (d, p) per frame."""
    ex = GpuExecutor(DEV, n_slots=slots, keep_outputs=True)
    srv = Server(ex, hbm_budget=1 << 40)
    ids = [srv.open_stream(StreamSpec(f[0][0].shape[1], f[0][0].shape[0], pipeline.camera_of(s), c))
           for s, f, m, c in streams]
    for i, k in order:
        s, f, m, c = streams[i]
        R, t = m[k] if k > 0 else (None, None)
        srv.submit(ids[i], f[k][0], f[k][1], R, t)
        srv.tick()
    srv.drain(timeout=120)
    torch.cuda.synchronize()
    out = {i: [] for i in range(len(streams))}
    for r in sorted(srv.results, key=lambda r: (r.sid, r.seq)):
        assert r.status == "ok"
        out[ids.index(r.sid)].append((r.d, r.p))
    return out


@pytest.mark.parametrize("slots", [1, 2])
def test_served_stream_is_the_same_alone_in_a_mix_and_in_the_pipeline(slots):
    _say("serving alone vs mix, slots", slots)
    cfg_a = pipeline.FrameConfig(max_disp=32, r_fixed=3)
    cfg_b = pipeline.FrameConfig(max_disp=16, r_fixed=-1, r_min=1, r_max=8)
    A = (*_sequence(128, 48, 4, 1), cfg_a)
    B = (*_sequence(96, 40, 4, 2), cfg_b)
    C = (*_sequence(128, 48, 4, 3), cfg_a)
    alone = _serve([A], [(0, k) for k in range(4)], slots)
    mix = _serve([B, A, C], [(0, 0), (1, 0), (2, 0), (2, 1), (1, 1), (0, 1), (1, 2), (0, 2),
                             (2, 2), (2, 3), (0, 3), (1, 3)], slots)
    # the plain per-frame pipeline with its own matcher
    st = pipeline.StreamState(128, 48, pipeline.camera_of(A[0]),
                              pipeline.FrameConfig(**{**cfg_a.__dict__, "overlap_census": True}), DEV)
    ref = []
    for k, (L, R) in enumerate(A[1]):
        Rm, t = A[2][k] if k > 0 else (None, None)
        d, p = st.step(L, R, Rm, t)
        ref.append((d.clone(), p.clone()))
    torch.cuda.synchronize()
    assert len(alone[0]) == len(mix[1]) == 4
    for k in range(4):
        for a, b, c in zip(alone[0][k], mix[1][k], ref[k]):
            assert torch.equal(a, b), k
            assert torch.equal(a, c), k
