"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Integer results (census codes, costs, path costs, aggregated costs, WTA and
right maps, LR decisions, windows, warp validity) must be bit-exact; float
results (subpixel, warp, Kalman) must be within 1e-4 px of the oracle's
double-precision values.  Inputs are seeded synthetic images; every case
prints its parameters before it runs.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_1708_06301_amd import egosgm as eg
from paper_1708_06301_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4
DEV = "cuda:0"


def _say(*a):
    print("CASE", *a, flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _random_pair(w, h, seed, max_shift=20):
    r = np.random.default_rng(seed)
    left = synth.texture(w, h, seed, noise_sigma=8.0, scale=5.0)
    shift = int(r.integers(0, max_shift + 1))
    right = np.roll(left, -shift, axis=1)
    right = np.clip(right.astype(int) + r.integers(-3, 4, size=right.shape), 0, 255).astype(np.uint8)
    return left, right


def _check_sgm(g, o, total, debug=True):
    assert np.array_equal(_np(g["disp_wta"]), o["disp_wta"])
    assert np.array_equal(_np(g["disp_right"]), o["disp_right"])
    assert np.array_equal(_np(g["var_meas"]).astype(np.float64), o["var_meas"])
    sub = _np(g["disp_sub"]).astype(np.float64)
    assert np.array_equal(sub < 0, o["disp_sub"] < 0)
    assert np.abs(sub - o["disp_sub"]).max() <= TOL
    if debug:
        assert np.array_equal(_np(g["wta_raw"]), o["wta_raw"])
        assert np.array_equal(_np(g["census_left"]).view(np.uint64), o["census_l"])
        assert np.array_equal(_np(g["census_right"]).view(np.uint64), o["census_r"])
        assert np.array_equal(_np(g["cost"])[:total].astype(np.int32), o["cost"])
        assert np.array_equal(_np(g["agg"])[:total].view(np.uint16).astype(np.int32), o["agg"])
        paths = _np(g["paths"])
        for k in range(8):
            assert np.array_equal(paths[k, :total].astype(np.int32), o["paths"][k]), f"path {k}"


@pytest.mark.parametrize("w,h", [(17, 9), (70, 13), (320, 96), (129, 7), (1, 1), (3, 2), (1242, 375)])
def test_census(w, h):
    _say("census", w, h)
    img = np.random.default_rng(w * h).integers(0, 256, size=(h, w)).astype(np.uint8)
    g = _np(eg.census(_gpu(img))).view(np.uint64)
    assert np.array_equal(g, orc.census(img))


@pytest.mark.parametrize("w,h,D", [(37, 19, 8), (53, 21, 24), (66, 17, 40), (70, 23, 64),
                                   (45, 30, 100), (70, 23, 128), (150, 9, 128), (290, 11, 256)])
def test_sgm_full_tiny(w, h, D):
    _say("sgm_full", w, h, D)
    left, right = _random_pair(w, h, seed=w + 100 * D, max_shift=min(D - 1, 20))
    prm = eg.MatchParams(max_disp=D, p1=7, p2=90, s_max=60, lr_tol=1)
    g = eg.sgm_full(_gpu(left), _gpu(right), prm, debug=True)
    o = orc.sgm(left, right, D, p1=7, p2=90, s_max=60, lr_tol=1, want_debug=True)
    _check_sgm(g, o, w * h * D)


def test_sgm_full_planes_config():
    _say("sgm_full planes 320x96 D=64")
    left, right, _ = synth.planes_pair()
    prm = eg.MatchParams(max_disp=64, p1=10, p2=120, s_max=80, lr_tol=1)
    g = eg.sgm_full(_gpu(left), _gpu(right), prm, debug=True)
    o = orc.sgm(left, right, 64, p1=10, p2=120, s_max=80, lr_tol=1, want_debug=True)
    _check_sgm(g, o, 320 * 96 * 64)


def _random_windows(w, h, D, seed, rmax=6, frac_full=0.1, kind="random"):
    """Predictions for ragged-window tests.  "random": independent centres
    (the window start moves at every step); "smooth": a slanted plane, so
    runs of equal window starts alternate with small moves; "wide": smooth
    with radii up to rmax (windows wider than 64)."""
    r = np.random.default_rng(seed)
    if kind == "random":
        d = r.uniform(0, D - 1, size=(h, w)).astype(np.float32)
    else:
        y, x = np.mgrid[0:h, 0:w]
        d = (0.2 * D + 0.04 * x + 0.25 * y + r.normal(0, 0.2, (h, w))).astype(np.float32)
        d = np.clip(d, 0, D - 1).astype(np.float32)
    d[r.random((h, w)) < frac_full] = -1.0
    p = r.uniform(0, (rmax / 3.0) ** 2, size=(h, w)).astype(np.float32)
    return d, p


@pytest.mark.parametrize("sched", [0, 1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("w,h,D,seed,kind,rmax", [
    (37, 19, 16, 1, "random", 6), (64, 20, 64, 2, "random", 6), (91, 27, 128, 3, "random", 6),
    (33, 5, 256, 4, "random", 6), (150, 23, 128, 5, "smooth", 6), (97, 17, 256, 6, "wide", 60),
    (80, 12, 64, 7, "wide", 40)])
def test_sgm_reduced_ragged(w, h, D, seed, kind, rmax, sched):
    _say("sgm_reduced", w, h, D, seed, kind, "schedule", sched)
    left, right = _random_pair(w, h, seed=seed + 7, max_shift=min(D - 1, 30))
    d, p = _random_windows(w, h, D, seed, rmax=rmax, kind=kind)
    r_max = max(12, rmax)
    lo, hi, off = eg.windows_from_prediction(_gpu(d), _gpu(p), D, r_min=0, r_max=r_max)
    wo = orc.windows(d, p, D, r_min=0, r_max=r_max)
    assert np.array_equal(_np(lo).ravel(), wo[0])
    assert np.array_equal(_np(hi).ravel(), wo[1])
    assert np.array_equal(_np(off).view(np.uint32), wo[2])
    prm = eg.MatchParams(max_disp=D, p1=10, p2=120, s_max=80, lr_tol=1)
    eg.set_tuning(**{**eg.DEFAULT_TUNING, "ragged_schedule": sched})
    try:
        g = eg.sgm_reduced(_gpu(left), _gpu(right), lo, hi, off, prm, debug=True)
    finally:
        eg.set_tuning(**eg.DEFAULT_TUNING)
    o = orc.sgm(left, right, D, windows=wo, want_debug=True)
    _check_sgm(g, o, int(wo[2][-1]))


@pytest.mark.parametrize("ragged,sched", [(False, 1), (True, 1), (True, 4), (True, 5), (True, 6), (True, 7), (True, 8)])
@pytest.mark.parametrize("D", [64, 100, 128])
def test_four_path_variant(ragged, sched, D):
    """n_paths = 4: directions 0-3 only (path volumes 0-3 and S bit-exact)."""
    _say("4 paths, ragged" if ragged else "4 paths, full", D, "schedule", sched)
    w, h = 91, 27
    left, right = _random_pair(w, h, seed=D + 3, max_shift=min(D - 1, 30))
    prm = eg.MatchParams(max_disp=D, p1=10, p2=120, s_max=40, lr_tol=1, n_paths=4)
    if ragged:
        d, p = _random_windows(w, h, D, seed=D + 4, kind="smooth")
        wo = orc.windows(d, p, D, r_min=0, r_max=12)
        lo, hi, off = (_gpu(wo[0].reshape(h, w)), _gpu(wo[1].reshape(h, w)), _gpu(wo[2].view(np.int32)))
        eg.set_tuning(ragged_schedule=sched)
        try:
            g = eg.sgm_reduced(_gpu(left), _gpu(right), lo, hi, off, prm, debug=True)
        finally:
            eg.set_tuning(**eg.DEFAULT_TUNING)
    else:
        wo = None
        g = eg.sgm_full(_gpu(left), _gpu(right), prm, debug=True)
    o = orc.sgm(left, right, D, p1=10, p2=120, s_max=40, lr_tol=1, windows=wo, want_debug=True,
                n_paths=4)
    total = int(wo[2][-1]) if ragged else w * h * D
    assert np.array_equal(_np(g["disp_wta"]), o["disp_wta"])
    assert np.array_equal(_np(g["disp_right"]), o["disp_right"])
    assert np.array_equal(_np(g["var_meas"]).astype(np.float64), o["var_meas"])
    assert np.abs(_np(g["disp_sub"]).astype(np.float64) - o["disp_sub"]).max() <= TOL
    assert np.array_equal(_np(g["agg"])[:total].view(np.uint16).astype(np.int32), o["agg"])
    paths = _np(g["paths"])
    for k in range(4):
        assert np.array_equal(paths[k, :total].astype(np.int32), o["paths"][k]), f"path {k}"


@pytest.mark.parametrize("sched", [1, 4, 6, 8])
@pytest.mark.parametrize("s_max", [0, 7, 80, 600])
@pytest.mark.parametrize("rmax,D", [(7, 64), (12, 128), (40, 128)])
def test_selection_walk_every_pixel(s_max, rmax, D, sched):
    """Left-right check off, so the uncertainty count and subpixel of every
    pixel are compared; windows up to 15 slots take the parallel walk, wider
    ones the serial one (schedule 1); schedule 4's selection takes windows
    whose quad span fits 16 slots in 4-lane groups, wider ones by the wave."""
    _say("selection walk, s_max", s_max, "rmax", rmax, "D", D, "schedule", sched)
    w, h = 83, 21
    left, right = _random_pair(w, h, seed=s_max + rmax, max_shift=min(D - 1, 30))
    d, p = _random_windows(w, h, D, seed=rmax + 5, rmax=rmax, kind="smooth", frac_full=0.05)
    wo = orc.windows(d, p, D, r_min=0, r_max=rmax)
    lo, hi, off = (_gpu(wo[0].reshape(h, w)), _gpu(wo[1].reshape(h, w)), _gpu(wo[2].view(np.int32)))
    prm = eg.MatchParams(max_disp=D, p1=10, p2=120, s_max=s_max, lr_tol=-1)
    eg.set_tuning(ragged_schedule=sched)
    try:
        g = eg.sgm_reduced(_gpu(left), _gpu(right), lo, hi, off, prm)
    finally:
        eg.set_tuning(**eg.DEFAULT_TUNING)
    o = orc.sgm(left, right, D, p1=10, p2=120, s_max=s_max, lr_tol=-1, windows=wo)
    assert np.array_equal(_np(g["disp_wta"]), o["disp_wta"])
    assert np.array_equal(_np(g["var_meas"]).astype(np.float64), o["var_meas"])
    assert np.abs(_np(g["disp_sub"]).astype(np.float64) - o["disp_sub"]).max() <= TOL


def test_census_on_another_stream_then_reduced():
    """sgm_census on a second stream, then sgm_reduced with census_ready=1
    on the first (ordered by an event), equals sgm_reduced alone."""
    _say("census ahead, 300x70 D=96")
    w, h, D = 300, 70, 96
    left, right = _random_pair(w, h, seed=77, max_shift=40)
    d, p = _random_windows(w, h, D, seed=78)
    lo, hi, off = eg.windows_from_prediction(_gpu(d), _gpu(p), D, r_min=1, r_max=6)
    L, R = _gpu(left), _gpu(right)
    ref = eg.sgm_reduced(L, R, lo, hi, off, eg.MatchParams(D))
    ws = eg.Workspace(DEV)
    side = torch.cuda.Stream(device=DEV)
    ev = torch.cuda.Event()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        eg.sgm_census(L, R, D, workspace=ws)
        ev.record(side)
    torch.cuda.current_stream().wait_event(ev)
    prm = eg.MatchParams(D)
    prm.census_ready = 1
    got = eg.sgm_reduced(L, R, lo, hi, off, prm, workspace=ws)
    torch.cuda.synchronize()
    for k in ("disp_wta", "disp_sub", "var_meas", "disp_right"):
        assert torch.equal(got[k], ref[k]), k


@pytest.mark.parametrize("D", [48, 128])
def test_sgm_reduced_full_windows_equal_full(D):
    _say("reduced == full, 120x40", D)
    left, right = _random_pair(120, 40, seed=17, max_shift=30)
    lo, hi, off = eg.windows_from_prediction(_gpu(np.full((40, 120), -1, np.float32)), None, D,
                                             r_fixed=3)
    prm = eg.MatchParams(max_disp=D)
    a = eg.sgm_reduced(_gpu(left), _gpu(right), lo, hi, off, prm, debug=True)
    b = eg.sgm_full(_gpu(left), _gpu(right), prm, debug=True)
    for k in ("disp_wta", "disp_sub", "var_meas", "disp_right", "agg", "paths"):
        assert torch.equal(a[k], b[k]), k


def test_windows_edge_values():
    _say("windows edge values")
    D = 128
    d = np.array([10.5, 10.499999, 1.0, -1.0, 200.0, np.nan, 0.0, 127.0, 126.5, 65536.0,
                  70000.0, -0.0, 3.5, 2.5], np.float32)
    p = np.array([1.0, 1.0000001, 0.0, 100.0, -1.0, np.inf, 4.0, 0.25, np.nan, 1, 1, 2.25,
                  1e-30, 1e30], np.float32)
    for r_fixed in (-1, 4):
        lo, hi, off = eg.windows_from_prediction(_gpu(d[None, :]), _gpu(p[None, :]), D,
                                                 r_fixed=r_fixed, r_min=1, r_max=16)
        wo = orc.windows(d, p, D, r_fixed=r_fixed, r_min=1, r_max=16)
        assert np.array_equal(_np(lo).ravel(), wo[0]) and np.array_equal(_np(hi).ravel(), wo[1])
        assert np.array_equal(_np(off).view(np.uint32), wo[2])
    r = np.random.default_rng(3)
    d = (r.integers(0, 300, 5000) / 2.0 + r.choice([0, 1e-6, -1e-6], 5000)).astype(np.float32)
    p = (r.integers(0, 30, 5000) ** 2 / 9.0 * r.choice([1, 1 + 1e-7, 1 - 1e-7], 5000)).astype(np.float32)
    lo, hi, off = eg.windows_from_prediction(_gpu(d.reshape(50, 100)), _gpu(p.reshape(50, 100)), D,
                                             r_min=0, r_max=40)
    wo = orc.windows(d, p, D, r_min=0, r_max=40)
    assert np.array_equal(_np(lo).ravel(), wo[0]) and np.array_equal(_np(hi).ravel(), wo[1])
    assert np.array_equal(_np(off).view(np.uint32), wo[2])


@pytest.mark.parametrize("w,h", [(256, 3), (257, 2), (513, 5), (700, 4), (1, 9), (300, 1100),
                                 (4000, 600)])
def test_windows_across_row_chunks(w, h):
    """Offsets are built per 256-pixel chunk of a row and then shifted by
    the earlier chunks' totals: widths on and around chunk boundaries, and
    more chunks than one pass of the totals' sum covers (2048)."""
    _say("windows chunks", w, h)
    D = 96
    r = np.random.default_rng(w * 7 + h)
    d = r.uniform(-5, 100, (h, w)).astype(np.float32)
    p = r.uniform(0, 30, (h, w)).astype(np.float32)
    for r_fixed in (-1, 3):
        lo, hi, off = eg.windows_from_prediction(_gpu(d), _gpu(p), D, r_fixed=r_fixed, r_min=0, r_max=40)
        wo = orc.windows(d.ravel(), p.ravel(), D, r_fixed=r_fixed, r_min=0, r_max=40)
        assert np.array_equal(_np(lo).ravel(), wo[0]) and np.array_equal(_np(hi).ravel(), wo[1])
        assert np.array_equal(_np(off).view(np.uint32), wo[2])


def _rot(a, b, c):
    ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
    return (np.array([[ca, 0, sa], [0, 1, 0], [-sa, 0, ca]]) @
            np.array([[1, 0, 0], [0, cb, -sb], [0, sb, cb]]) @
            np.array([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]]))


def _close(g, o):
    """|g - o| within 1e-4 px, or half a float32 ulp of o where that is larger
    (only for values above 2048, far outside any disparity range)."""
    tol = np.maximum(TOL, 0.5 * np.spacing(np.abs(o).astype(np.float32)).astype(np.float64))
    return bool((np.abs(g.astype(np.float64) - o) <= tol).all())


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_warp(seed):
    r = np.random.default_rng(seed)
    w, h = (1242, 375) if seed == 0 else (int(r.integers(20, 300)), int(r.integers(10, 120)))
    _say("warp", w, h, seed)
    d = r.uniform(0.5, 120, size=(h, w)).astype(np.float32)
    d[r.random((h, w)) < 0.1] = -1.0
    p = r.uniform(0.01, 6, size=(h, w)).astype(np.float32)
    R = _rot(*r.normal(0, 0.01, 3))
    t = np.array([r.normal(0, 0.05), r.normal(0, 0.02), -abs(r.normal(1.0, 0.2))])
    f = 718.0 * w / 1242.0
    cam = (f, (w - 1) / 2, (h - 1) / 2, 0.54)
    H = eg.warp_matrix(R, t, *cam)
    Ho = orc.warp_matrix(R, t, *cam).astype(np.float32)
    assert np.array_equal(H, Ho)
    gd, gp = eg.warp_disparity(_gpu(d), _gpu(p), R, t, *cam, 0.5)
    o = orc.warp(d, p, R, t, *cam, q=0.5)
    gd, gp = _np(gd), _np(gp)
    valid = o["winner"] >= 0
    assert np.array_equal(gd >= 0, valid)
    assert _close(gd[valid], o["d_pred"][valid])
    assert _close(gp[valid], o["p_pred"][valid])
    assert (gd[~valid] == -1).all() and (gp[~valid] == 0).all()


def test_warp_identity_and_collisions():
    _say("warp identity")
    r = np.random.default_rng(9)
    d = r.uniform(1, 50, size=(31, 77)).astype(np.float32)
    p = r.uniform(0, 3, size=(31, 77)).astype(np.float32)
    gd, gp = eg.warp_disparity(_gpu(d), _gpu(p), np.eye(3), np.zeros(3), 300.0, 38.0, 15.0, 0.5, 0.25)
    assert np.array_equal(_np(gd), d) and np.array_equal(_np(gp), p + np.float32(0.25))
    # many sources per target: strong backward motion contracts the image
    d = np.full((40, 60), 20.0, np.float32) + r.uniform(0, 1, (40, 60)).astype(np.float32)
    d[:, ::7] = 20.0  # exact ties between sources
    p = r.uniform(0, 3, size=(40, 60)).astype(np.float32)
    cam = (100.0, 29.5, 19.5, 0.5)
    t = np.array([0.0, 0.0, 5.0])
    gd, gp = eg.warp_disparity(_gpu(d), _gpu(p), np.eye(3), t, *cam, 0.5)
    o = orc.warp(d, p, np.eye(3), t, *cam, q=0.5)
    gd, gp = _np(gd), _np(gp)
    assert np.array_equal(gd >= 0, o["winner"] >= 0)
    assert _close(gd, o["d_pred"]) and _close(gp, o["p_pred"])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_refine(seed):
    r = np.random.default_rng(50 + seed)
    h, w = (375, 1242) if seed == 0 else (int(r.integers(5, 90)), int(r.integers(5, 200)))
    _say("refine", w, h, seed)
    base = np.cumsum(r.normal(0, 0.4, size=(h, w)), axis=1).astype(np.float32) + 40
    d = np.where(r.random((h, w)) < 0.3, -1.0, base).astype(np.float32)
    d[r.random((h, w)) < 0.02] += 10.0
    p = r.uniform(0.1, 4, size=(h, w)).astype(np.float32)
    for edge_tol, fill_tol in ((-1.0, 1.0), (2.0, 1.0), (0.5, 0.0), (3.0, 2.5), (0.0, 0.25)):
        gd, gp = eg.refine_prediction(_gpu(d), _gpu(p), edge_tol, fill_tol)
        od, op = orc.refine(d, p, edge_tol, fill_tol)
        assert np.array_equal(_np(gd), od) and np.array_equal(_np(gp), op), (edge_tol, fill_tol)


@pytest.mark.parametrize("h,w", [(1, 1), (1, 7), (5, 1), (2, 3), (3, 65), (9, 2)])
def test_refine_degenerate_shapes(h, w):
    _say("refine degenerate", w, h)
    r = np.random.default_rng(h * 100 + w)
    d = np.where(r.random((h, w)) < 0.4, -1.0, r.uniform(10, 12, (h, w))).astype(np.float32)
    p = r.uniform(0.1, 4, size=(h, w)).astype(np.float32)
    for edge_tol, fill_tol in ((-1.0, 1.0), (1.0, 3.0), (0.0, 0.0)):
        gd, gp = eg.refine_prediction(_gpu(d), _gpu(p), edge_tol, fill_tol)
        od, op = orc.refine(d, p, edge_tol, fill_tol)
        assert np.array_equal(_np(gd), od) and np.array_equal(_np(gp), op), (edge_tol, fill_tol)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_predict_disparity_equals_warp_then_refine(seed):
    """The fused prediction decodes the z-buffer inside the refinement; its
    maps must be bit-identical to warp_disparity followed by refine_prediction."""
    r = np.random.default_rng(70 + seed)
    w, h = (1242, 375) if seed == 0 else (int(r.integers(3, 300)), int(r.integers(2, 120)))
    _say("predict fused", w, h, seed)
    base = np.cumsum(r.normal(0, 0.3, size=(h, w)), axis=1).astype(np.float32) + 30
    d = np.where(r.random((h, w)) < 0.1, -1.0, base).astype(np.float32)
    p = r.uniform(0.01, 5, size=(h, w)).astype(np.float32)
    R = _rot(*r.normal(0, 0.01, 3))
    t = np.array([r.normal(0, 0.05), r.normal(0, 0.02), -abs(r.normal(1.0, 0.2))])
    f = 718.0 * w / 1242.0
    cam = (f, (w - 1) / 2, (h - 1) / 2, 0.54)
    for edge_tol, fill_tol in ((2.0, 1.0), (-1.0, 0.0), (0.5, 3.0)):
        gd, gp = eg.warp_disparity(_gpu(d), _gpu(p), R, t, *cam, 0.5)
        rd, rp = eg.refine_prediction(gd, gp, edge_tol, fill_tol)
        fd, fp = eg.predict_disparity(_gpu(d), _gpu(p), R, t, *cam, 0.5, edge_tol, fill_tol)
        assert np.array_equal(_np(fd), _np(rd)) and np.array_equal(_np(fp), _np(rp)), (edge_tol, fill_tol)


@pytest.mark.parametrize("n", [100003, 1, 255, 1025, 4 * 256 + 3])
def test_kalman(n):
    """Sizes around one block's kEw * 256 pixels and a ragged tail."""
    _say("kalman", n)
    r = np.random.default_rng(4)
    dp = r.uniform(0, 255, n).astype(np.float32)
    pp = r.uniform(0.001, 100, n).astype(np.float32)
    z = (dp + r.normal(0, 3, n)).astype(np.float32)
    rr = r.integers(0, 60, n).astype(np.float32)
    dp[r.random(n) < 0.1] = -1
    z[r.random(n) < 0.1] = -1
    pp[r.random(n) < 0.02] = 0
    for keep in (0, 1):
        gd, gp = eg.kalman_update(*[_gpu(a) for a in (dp, pp, z, rr)], keep_unmeasured=keep)
        od, op = orc.kalman(dp, pp, z, rr, keep)
        gd, gp = _np(gd), _np(gp)
        assert np.array_equal(gd < 0, od < 0)
        assert np.abs(gd - od).max() <= TOL and np.abs(gp - op).max() <= TOL


@pytest.mark.parametrize("D", [64, 128, 256])
def test_tuning_never_changes_results(D):
    _say("tuning invariance", D)
    import itertools
    w, h = 97, 29
    left, right = _random_pair(w, h, seed=D, max_shift=min(D - 1, 40))
    d, p = _random_windows(w, h, D, seed=D + 1, frac_full=0.15)
    wo = orc.windows(d, p, D, r_min=0, r_max=12)
    o_full = orc.sgm(left, right, D)
    o_red = orc.sgm(left, right, D, windows=wo)
    L, R = _gpu(left), _gpu(right)
    lo, hi, off = (_gpu(wo[0].reshape(h, w)), _gpu(wo[1].reshape(h, w)),
                   _gpu(wo[2].view(np.int32)))
    prm = eg.MatchParams(max_disp=D)
    try:
        # wide_offsets = 1 runs the 64-bit addressing that images of 2^27 pixels take
        for fg, rg, pr, wo_ in itertools.product((16, 32, 64), (16, 32, 64), (0, 1, 2, 3, 4, 5, 6, 7, 8), (0, 1)):
            eg.set_tuning(fg, rg, pr, wide_offsets=wo_)
            a = eg.sgm_full(L, R, prm)
            b = eg.sgm_reduced(L, R, lo, hi, off, prm)
            assert np.array_equal(_np(a["disp_wta"]), o_full["disp_wta"]), (fg, rg, pr, wo_)
            assert np.array_equal(_np(a["var_meas"]).astype(np.float64), o_full["var_meas"])
            assert np.array_equal(_np(b["disp_wta"]), o_red["disp_wta"]), (fg, rg, pr, wo_)
            assert np.array_equal(_np(b["disp_right"]), o_red["disp_right"]), (fg, rg, pr, wo_)
    finally:
        eg.set_tuning(**eg.DEFAULT_TUNING)


# ---------------------------------------------------------------- batches
def _batch_cases():
    specs = [(37, 19, 16, False), (64, 20, 64, True), (91, 27, 128, True), (45, 30, 100, False),
             (70, 23, 128, True), (130, 9, 256, True), (33, 41, 48, False)]
    cases = []
    for i, (w, h, D, ragged) in enumerate(specs):
        left, right = _random_pair(w, h, seed=300 + i, max_shift=min(D - 1, 30))
        win = None
        if ragged:
            d, p = _random_windows(w, h, D, seed=400 + i, frac_full=0.12)
            wo = orc.windows(d, p, D, r_min=0, r_max=12)
            win = (_gpu(wo[0].reshape(h, w)), _gpu(wo[1].reshape(h, w)), _gpu(wo[2].view(np.int32)))
        cases.append(dict(left=_gpu(left), right=_gpu(right), max_disp=D, windows=win))
    return cases


def _single(case, prm):
    p = eg.MatchParams(case["max_disp"], prm.p1, prm.p2, prm.s_max, prm.lr_tol, prm.n_paths)
    if case["windows"] is None:
        return eg.sgm_full(case["left"], case["right"], p)
    return eg.sgm_reduced(case["left"], case["right"], *case["windows"], p)


def _same(a, b):
    for k in ("disp_wta", "disp_sub", "var_meas", "disp_right"):
        if not torch.equal(a[k], b[k]):
            return k
    return None


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("group,n_paths", [(16, 8), (32, 8), (64, 8), (16, 4)])
def test_plan_matches_single_pairs(group, n_paths, persistent):
    _say("plan of 7 mixed pairs, lanes per scanline", group, "paths", n_paths, "persistent", persistent)
    cases = _batch_cases()
    prm = eg.MatchParams(max_disp=256, p1=9, p2=110, s_max=70, lr_tol=1, n_paths=n_paths)
    eg.set_tuning(**{**eg.DEFAULT_TUNING, "batch_group": group, "batch_persistent": persistent})
    try:
        plan = eg.Plan(cases, prm)
    finally:
        eg.set_tuning(**eg.DEFAULT_TUNING)
    plan.run()
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        ref = _single(c, prm)
        torch.cuda.synchronize()
        assert _same(plan.outputs[i], ref) is None, (i, _same(plan.outputs[i], ref))
    # every pair also against the oracle, every output
    for i, c in enumerate(cases):
        wo = None
        if c["windows"] is not None:
            wo = (c["windows"][0].cpu().numpy().ravel(), c["windows"][1].cpu().numpy().ravel(),
                  c["windows"][2].cpu().numpy().view(np.uint32))
        o = orc.sgm(c["left"].cpu().numpy(), c["right"].cpu().numpy(), c["max_disp"], prm.p1, prm.p2,
                    prm.s_max, prm.lr_tol, windows=wo, n_paths=n_paths)
        g = plan.outputs[i]
        assert np.array_equal(_np(g["disp_wta"]), o["disp_wta"]), i
        assert np.array_equal(_np(g["disp_right"]), o["disp_right"]), i
        assert np.array_equal(_np(g["var_meas"]).astype(np.float64), o["var_meas"]), i
        sub = _np(g["disp_sub"]).astype(np.float64)
        assert np.array_equal(sub < 0, o["disp_sub"] < 0), i
        assert np.abs(sub - o["disp_sub"]).max() <= TOL, i
    plan.close()


@pytest.mark.parametrize("persistent", [0, 1])
def test_plan_graph_replays_and_window_updates(persistent):
    _say("plan replays, persistent", persistent)
    cases = _batch_cases()[:4]
    prm = eg.MatchParams()
    eg.set_tuning(**{**eg.DEFAULT_TUNING, "batch_persistent": persistent})
    try:
        plan = eg.Plan(cases, prm)
    finally:
        eg.set_tuning(**eg.DEFAULT_TUNING)
    refs = [_single(c, prm) for c in cases]
    for rep in range(3):
        for o in plan.outputs:
            for t in o.values():
                t.fill_(7)
        plan.run()
        x = torch.randn(1000, device=DEV).sum()   # eager work between replays
        torch.cuda.synchronize()
        for i in range(len(cases)):
            assert _same(plan.outputs[i], refs[i]) is None, (rep, i)
    # rewrite the ragged windows in place and replay
    c = cases[1]
    h, w = c["left"].shape
    d, p = _random_windows(w, h, 64, seed=999, frac_full=0.3)
    wo = orc.windows(d, p, 64, r_min=0, r_max=6)
    c["windows"][0].copy_(_gpu(wo[0].reshape(h, w)))
    c["windows"][1].copy_(_gpu(wo[1].reshape(h, w)))
    c["windows"][2].copy_(_gpu(wo[2].view(np.int32)))
    plan.run()
    ref = _single(c, prm)
    torch.cuda.synchronize()
    assert _same(plan.outputs[1], ref) is None
    del x
    plan.close()


# ---------------------------------------------------------------- full size
def test_street_frames_full_size_default_launch():
    """1242x375, D=128 in the default launch tuning (the bench's): frame 0
    over the full range and frame 1 through the pipeline's prediction,
    refinement and r=4 windows; the oracle gets the GPU's refined
    prediction, so windows and matcher outputs must agree exactly."""
    from paper_1708_06301_amd import pipeline
    _say("street frames 1242x375 D=128, default tuning")
    eg.set_tuning(**eg.DEFAULT_TUNING)
    w, h, D = 1242, 375, 128
    seq = synth.street_sequence(w, h, 2, seed=synth.seed_for(1))
    (L0, R0, _), (L1, R1, _) = seq.frame(0, device=DEV), seq.frame(1, device=DEV)
    cfg = pipeline.FrameConfig(max_disp=D, r_fixed=4)
    st = pipeline.StreamState(w, h, pipeline.camera_of(seq), cfg, DEV)
    st.step(_gpu(L0), _gpu(R0))
    torch.cuda.synchronize()
    o0 = orc.sgm(L0, R0, D, p1=cfg.p1, p2=cfg.p2, s_max=cfg.s_max, lr_tol=cfg.lr_tol)
    assert np.array_equal(_np(st.out["disp_wta"]), o0["disp_wta"])
    assert np.array_equal(_np(st.out["disp_right"]), o0["disp_right"])
    assert np.array_equal(_np(st.out["var_meas"]).astype(np.float64), o0["var_meas"])
    assert np.abs(_np(st.out["disp_sub"]).astype(np.float64) - o0["disp_sub"]).max() <= TOL
    Rm, t = (np.asarray(a, np.float64) for a in seq.motion(1))
    win = st.predict(Rm, t)
    st.match(_gpu(L1), _gpu(R1), win)
    torch.cuda.synchronize()
    wo = orc.windows(_np(st.d_pred), _np(st.p_pred), D, r_fixed=4, r_min=cfg.r_min, r_max=cfg.r_max)
    assert np.array_equal(_np(win[0]).ravel(), wo[0])
    assert np.array_equal(_np(win[1]).ravel(), wo[1])
    assert np.array_equal(_np(win[2]).view(np.uint32), wo[2])
    o1 = orc.sgm(L1, R1, D, p1=cfg.p1, p2=cfg.p2, s_max=cfg.s_max, lr_tol=cfg.lr_tol, windows=wo)
    assert np.array_equal(_np(st.out["disp_wta"]), o1["disp_wta"])
    assert np.array_equal(_np(st.out["disp_right"]), o1["disp_right"])
    assert np.array_equal(_np(st.out["var_meas"]).astype(np.float64), o1["var_meas"])
    assert np.abs(_np(st.out["disp_sub"]).astype(np.float64) - o1["disp_sub"]).max() <= TOL



@pytest.mark.parametrize("radius,sad_max", [(0, 5), (1, 60), (2, 300), (3, 900)])
def test_sad_check(radius, sad_max):
    _say("sad check", radius, sad_max)
    w, h, D = 97, 31, 64
    left, right = _random_pair(w, h, seed=radius + 50, max_shift=30)
    o = orc.sgm(left, right, D, lr_tol=-1)
    L, R = _gpu(left), _gpu(right)
    out = dict(disp_wta=_gpu(o["disp_wta"]), disp_sub=_gpu(o["disp_sub"].astype(np.float32)),
               var_meas=_gpu(o["var_meas"].astype(np.float32)))
    eg.sad_check(L, R, out, radius, sad_max)
    wta, sub, var = orc.sad_check(left, right, o["disp_wta"], radius, sad_max,
                                  o["disp_sub"].astype(np.float32), o["var_meas"].astype(np.float32))
    assert np.array_equal(_np(out["disp_wta"]), wta)
    assert np.array_equal(_np(out["disp_sub"]).astype(np.float64), sub)
    assert np.array_equal(_np(out["var_meas"]).astype(np.float64), var)
    assert 0 < (wta < 0).sum() < wta.size or radius == 0


def test_lr_check_prediction_and_float_maps():
    _say("lr check of a prediction, 211x57")
    r = np.random.default_rng(77)
    h, w = 57, 211
    d = r.uniform(0, 60, size=(h, w)).astype(np.float32)
    d[r.random((h, w)) < 0.1] = -1.0
    d[:, :3] = 50.0                       # references left of the image
    d[0, 10] = 9.5                        # rounds to 10: x - 10 = 0 is inside
    p = r.uniform(0.1, 4, size=(h, w)).astype(np.float32)
    dr = np.full((h, w), -1.0, np.float32)
    for y in range(h):                    # half of the pixels near agreement, the rest noise
        for x in range(w):
            if d[y, x] >= 0 and r.random() < 0.5:
                xr = x - int(np.floor(d[y, x] + 0.5))
                if xr >= 0:
                    dr[y, xr] = d[y, x] + (0.0 if r.random() < 0.3 else r.uniform(-1.5, 1.5))
    holes = dr < 0
    dr[holes] = np.where(r.random(holes.sum()) < 0.5, -1.0, r.uniform(0, 60, holes.sum())).astype(np.float32)
    for tol in (0.0, 0.5, 1.0, 2.0):
        gd, gp = _gpu(d), _gpu(p)
        eg.lr_check_prediction(gd, gp, _gpu(dr), tol)
        od, op = orc.lr_check_prediction(d, p, dr, tol)
        assert np.array_equal(_np(gd), od) and np.array_equal(_np(gp), op), tol
        kept = od >= 0
        assert 0 < kept.sum() < (d >= 0).sum()
    i16 = r.integers(-1, 128, size=(h, w)).astype(np.int16)
    out = torch.empty((h, w), dtype=torch.float32, device=DEV)
    eg.disparity_to_float(_gpu(i16), out)
    assert np.array_equal(_np(out), i16.astype(np.float32))


def test_prediction_with_lr_check_follows_the_oracle():
    """The pipeline's prediction with the left-right check on: the right
    map kept from frame 0 equals the matcher's, its warp with the right
    camera's motion matches the oracle's, and the checked left prediction
    equals the oracle's check of the unchecked one against the GPU's
    refined right prediction."""
    from paper_1708_06301_amd import pipeline
    _say("prediction lr check, street 320x96")
    w, h, D = 320, 96, 64
    seq = synth.street_sequence(w, h, 2, seed=synth.seed_for(2))
    (L0, R0, _), = [seq.frame(0, device=DEV)]
    Rm, t = (np.asarray(a, np.float64) for a in seq.motion(1))
    states = []
    for lr in (False, True):
        cfg = pipeline.FrameConfig(max_disp=D, r_fixed=4, lr_predict=lr, lr_predict_tol=1.0)
        st = pipeline.StreamState(w, h, pipeline.camera_of(seq), cfg, DEV)
        st.step(_gpu(L0), _gpu(R0))
        st.predict(Rm, t)
        states.append(st)
    off, on = states
    c = pipeline.camera_of(seq)
    assert np.array_equal(_np(on.d_r), _np(on.out["disp_right"]).astype(np.float32))
    tr = orc.right_motion(Rm, t, c.baseline)
    o = orc.warp(_np(on.d_r), np.zeros((h, w), np.float32), Rm, tr, c.f, c.cx, c.cy, c.baseline,
                 q=on.cfg.q)
    gd = _np(on.d_rwarp)
    valid = o["winner"] >= 0
    assert np.array_equal(gd >= 0, valid) and _close(gd[valid], o["d_pred"][valid])
    rd, rp = orc.refine(gd, _np(on.p_rwarp), on.cfg.edge_tol, on.cfg.fill_tol)
    assert np.array_equal(_np(on.d_rpred), rd) and np.array_equal(_np(on.p_rpred), rp)
    od, op = orc.lr_check_prediction(_np(off.d_pred), _np(off.p_pred), rd, on.cfg.lr_predict_tol)
    assert np.array_equal(_np(on.d_pred), od) and np.array_equal(_np(on.p_pred), op)
    n_off, n_on = int((_np(off.d_pred) >= 0).sum()), int((od >= 0).sum())
    assert 0.5 * n_off < n_on < n_off
