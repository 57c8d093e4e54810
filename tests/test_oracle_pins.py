"""Pins of the CPU oracle against facts fixed outside it.

Every check here compares the oracle with something other than itself:
hand-worked fixtures (tests/golden/), brute force over all disparity
sequences (the Viterbi form of the SGM path minimisation), closed forms
(Euclidean reprojection for the disparity-space warp, the algebraic form of
the Kalman update), special cases that collapse to a simpler rule, and
invariants of the definitions.
"""
import itertools

import numpy as np
import pytest

from golden_io import load
from paper_1708_06301_amd import synth


# ---------------------------------------------------------------- census
def test_census_golden(orc):
    g = load("census_hand.txt")
    img = np.array(g["image"], np.uint8)
    assert img.shape == (7, 9)
    c = orc.census(img)
    ci = orc.census(255 - img)
    assert int(c[3, 4]) == g["code_centre"]
    assert int(ci[3, 4]) == g["code_centre_inverted"]
    assert orc.cost(c, ci, 4, 3, 0) == g["hamming"]
    both = int(c[3, 4]) | int(ci[3, 4])
    assert 62 - bin(both).count("1") == g["ties"]


def test_census_constant_image_is_zero(orc):
    assert not orc.census(np.full((11, 13), 77, np.uint8)).any()


def test_census_raster_increasing_closed_form(orc):
    # With I(x,y) strictly increasing in raster order, "darker" means
    # "earlier in raster order", so each bit is a comparison of (clamped)
    # coordinates, not of intensities.
    w, h = 12, 9
    img = np.arange(w * h, dtype=np.uint8).reshape(h, w)
    c = orc.census(img)
    for y in range(h):
        for x in range(w):
            k, code = 0, 0
            for dy in range(-3, 4):
                for dx in range(-4, 5):
                    if dx == 0 and dy == 0:
                        continue
                    qy, qx = min(max(y + dy, 0), h - 1), min(max(x + dx, 0), w - 1)
                    if (qy, qx) < (y, x):
                        code |= 1 << k
                    k += 1
            assert int(c[y, x]) == code, (x, y)
    # interior pixels: exactly the 31 offsets before the centre
    assert int(c[4, 6]) == (1 << 31) - 1


def test_census_complement_and_ties(orc):
    r = np.random.default_rng(5)
    img = r.integers(0, 6, size=(10, 14)).astype(np.uint8)   # many ties
    a, b = orc.census(img), orc.census(255 - img)
    assert not (a & b).any()
    assert int(np.max(a)) < (1 << 62) and int(np.max(b)) < (1 << 62)
    # bits in neither code are exactly the neighbours equal to the centre
    y, x = 5, 7
    eq = sum(int(img[min(max(y + dy, 0), 9), min(max(x + dx, 0), 13)] == img[y, x])
             for dy in range(-3, 4) for dx in range(-4, 5) if (dx, dy) != (0, 0))
    assert 62 - bin(int(a[y, x]) | int(b[y, x])).count("1") == eq


def test_census_shift_equivariance(orc):
    r = np.random.default_rng(6)
    img = r.integers(0, 256, size=(20, 30)).astype(np.uint8)
    sh = np.roll(img, (2, 3), axis=(0, 1))
    a, b = orc.census(img), orc.census(sh)
    # away from borders and from the wrapped band the codes move with the image
    assert np.array_equal(b[2 + 3:20 - 3, 3 + 4:30 - 4], a[3:20 - 3 - 2, 4:30 - 4 - 3])


def test_cost_rules(orc):
    r = np.random.default_rng(7)
    img = r.integers(0, 256, size=(9, 16)).astype(np.uint8)
    c = orc.census(img)
    assert orc.cost(c, c, 10, 4, 0) == 0
    assert orc.cost(c, c, 3, 4, 4) == 62          # x - d < 0
    assert orc.cost(c, c, 3, 4, 3) == bin(int(c[4, 3]) ^ int(c[4, 0])).count("1")


# ---------------------------------------------------------------- paths
def _full(n, D):
    lo = np.zeros(n, np.int16)
    hi = np.full(n, D - 1, np.int16)
    off = np.arange(n + 1, dtype=np.uint32) * D
    return lo, hi, off


def test_path_golden(orc):
    g = load("path_hand.txt")
    cost = np.array(g["cost"], np.int32).ravel()
    lo, hi, off = _full(3, 3)
    for k in (0, 1):
        L = orc.path(cost, 3, 1, lo, hi, off, g["p1"], g["p2"], k)
        assert np.array_equal(L.reshape(3, 3), np.array(g[f"L_dir{k}"])), k
    # a 1-row image has no vertical or diagonal predecessors: L = C
    for k in range(2, 8):
        assert np.array_equal(orc.path(cost, 3, 1, lo, hi, off, g["p1"], g["p2"], k), cost)
    rl = np.array(g["ragged_lo"], np.int16)
    rh = np.array(g["ragged_hi"], np.int16)
    roff = np.concatenate([[0], np.cumsum(rh - rl + 1)]).astype(np.uint32)
    full = np.array(g["cost"])
    rc = np.concatenate([full[x, rl[x]:rh[x] + 1] for x in range(3)]).astype(np.int32)
    L = orc.path(rc, 3, 1, rl, rh, roff, g["p1"], g["p2"], 0)
    assert L.tolist() == g["ragged_L_dir0"]


def _scanlines(w, h, dx, dy):
    lines = []
    for y in range(h):
        for x in range(w):
            if 0 <= x - dx < w and 0 <= y - dy < h:
                continue
            line = []
            cx, cy = x, y
            while 0 <= cx < w and 0 <= cy < h:
                line.append(cy * w + cx)
                cx += dx
                cy += dy
            lines.append(line)
    return lines


def _viterbi_L(costs, wins, p1, p2):
    """Brute force: minimal energy over every disparity sequence along one
    scanline, E = sum C_i(d_i) + sum V(d_i, d_{i-1}), V in {0, P1, P2};
    then L_n(d) = E*_n(d) - min_k E*_{n-1}(k)."""
    def V(a, b):
        return 0 if a == b else (p1 if abs(a - b) == 1 else p2)

    out = []
    prev_min = None
    for n in range(len(costs)):
        best = {}
        for seq in itertools.product(*[range(lo, hi + 1) for lo, hi in wins[:n + 1]]):
            e = sum(costs[i][seq[i] - wins[i][0]] for i in range(n + 1))
            e += sum(V(seq[i], seq[i - 1]) for i in range(1, n + 1))
            best[seq[-1]] = min(best.get(seq[-1], 1 << 30), e)
        row = [best[d] - (prev_min if n else 0) for d in range(wins[n][0], wins[n][1] + 1)]
        prev_min = min(best.values())
        out.append(row)
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_path_matches_viterbi_bruteforce(orc, seed):
    r = np.random.default_rng(100 + seed)
    w, h, D = 4, 3, 4
    n = w * h
    lo = r.integers(0, D, size=n)
    hi = np.minimum(D - 1, lo + r.integers(0, D, size=n))
    if seed == 0:
        lo[:], hi[:] = 0, D - 1
    lo, hi = lo.astype(np.int16), hi.astype(np.int16)
    off = np.concatenate([[0], np.cumsum(hi - lo + 1)]).astype(np.uint32)
    cost = r.integers(0, 63, size=int(off[-1])).astype(np.int32)
    p1 = int(r.integers(0, 15))
    p2 = p1 + int(r.integers(0, 40))
    for k in range(8):
        dx, dy = orc.direction(k)
        L = orc.path(cost, w, h, lo, hi, off, p1, p2, k)
        for line in _scanlines(w, h, dx, dy):
            costs = [cost[off[p]:off[p + 1]].tolist() for p in line]
            wins = [(int(lo[p]), int(hi[p])) for p in line]
            ref = _viterbi_L(costs, wins, p1, p2)
            for p, row in zip(line, ref):
                assert L[off[p]:off[p + 1]].tolist() == row, (k, p)


def test_directions_cover_the_eight_neighbours(orc):
    dirs = {orc.direction(k) for k in range(8)}
    assert dirs == {(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)} - {(0, 0)}


def test_sgm_zero_penalties_reduce_to_cost(orc):
    left, right, _ = synth.planes_pair(64, 24, seed=11)
    r = orc.sgm(left, right, 16, p1=0, p2=0, lr_tol=-1, want_debug=True)
    cost = r["cost"].reshape(24, 64, 16)
    for k in range(8):
        assert np.array_equal(r["paths"][k], r["cost"])
    assert np.array_equal(r["agg"], 8 * r["cost"])
    assert np.array_equal(r["disp_wta"], np.argmin(cost, axis=2))


def test_four_path_variant_sums_the_axis_directions(orc):
    """4 paths = directions 0-3 (along and against rows and columns); with
    zero penalties S = 4C, and in general S is the sum of those four
    single-direction volumes, each of which the Viterbi pins fix."""
    left, right, _ = synth.planes_pair(64, 24, seed=13)
    z = orc.sgm(left, right, 16, p1=0, p2=0, lr_tol=-1, want_debug=True, n_paths=4)
    assert z["paths"].shape[0] == 4
    assert np.array_equal(z["agg"], 4 * z["cost"])
    r8 = orc.sgm(left, right, 16, p1=10, p2=120, want_debug=True)
    r4 = orc.sgm(left, right, 16, p1=10, p2=120, want_debug=True, n_paths=4)
    assert [orc.direction(k) for k in range(4)] == [(1, 0), (-1, 0), (0, 1), (0, -1)]
    assert np.array_equal(r4["paths"], r8["paths"][:4])
    assert np.array_equal(r4["agg"], r8["paths"][:4].sum(axis=0))
    S = r4["agg"].reshape(24, 64, 16)
    assert np.array_equal(r4["wta_raw"], np.argmin(S, axis=2))


def test_sgm_bounds_and_sum(orc):
    left, right, _ = synth.planes_pair(48, 20, seed=12)
    r = orc.sgm(left, right, 24, p1=10, p2=120, want_debug=True)
    assert r["paths"].min() >= 0 and r["paths"].max() <= 62 + 120
    assert np.array_equal(r["paths"].sum(axis=0), r["agg"])


@pytest.mark.parametrize("d0", [0, 5, 13])
def test_sgm_fronto_parallel_plane_exact(orc, d0):
    w, h, D = 72, 26, 24
    left, right = synth.shifted_pair(w, h, d0, seed=21 + d0)
    r = orc.sgm(left, right, D, p1=10, p2=120, lr_tol=1)
    interior = (slice(0, h), slice(d0 + 8, w - 8))
    assert (r["disp_wta"][interior] == d0).all()
    assert (r["disp_right"][:, 8:w - d0 - 8] == d0).all()
    assert (np.abs(r["disp_sub"][interior] - d0) < 0.5).all()


def test_sgm_planes_accuracy(orc):
    # c1-shaped pair: the disparity field is known in right-image coordinates,
    # so compare through the right map's interior.
    left, right, d_right = synth.planes_pair(160, 48, seed=13, integer=True, noise_sigma=3.0)
    r = orc.sgm(left, right, 64)
    good = np.abs(r["disp_right"][:, 8:-70].astype(np.float64) - d_right[:, 8:-70]) <= 1
    assert good.mean() > 0.9


# ---------------------------------------------------------------- epilogue
def test_epilogue_golden(orc):
    for (lo, hi, s_max), S, (ds, sub, nl, nr) in load("epilogue_hand.txt")["case"]:
        got = orc.pixel_epilogue(np.array(S), lo, hi, s_max)
        assert got[0] == ds and got[2] == nl and got[3] == nr
        assert got[1] == pytest.approx(sub, abs=1e-12)


def test_epilogue_limits(orc):
    r = np.random.default_rng(8)
    for _ in range(50):
        lo = int(r.integers(0, 50))
        S = r.integers(0, 1400, size=int(r.integers(1, 40)))
        hi = lo + S.size - 1
        ds, sub, nl, nr = orc.pixel_epilogue(S, lo, hi, 1 << 30)
        assert S[ds - lo] == S.min() and ds - lo == int(np.argmin(S))
        assert (nl, nr) == (ds - lo, hi - ds)           # S_max -> infinity
        assert orc.pixel_epilogue(S, lo, hi, 0)[2:] == (0, 0)
        assert abs(sub - ds) <= 0.5
    # symmetric neighbours: no offset
    assert orc.pixel_epilogue(np.array([9, 2, 9]), 0, 2, 10)[1] == 1.0


# ---------------------------------------------------------------- right map / LR
def test_right_map_and_lr_golden(orc):
    g = load("rightdm_hand.txt")
    S = np.array(g["S"], np.int32)
    lo, hi, off = _full(4, 3)
    dr = orc.right_map(S.ravel(), 4, 1, 3, lo, hi, off)
    assert dr.ravel().tolist() == g["right"]
    wta = np.array([[int(np.argmin(S[x])) for x in range(4)]], np.int16)
    assert wta.ravel().tolist() == g["wta"]
    for tol in (1, 0):
        got, _, _ = orc.lr_check(dr, wta, tol)
        assert got.ravel().tolist() == g[f"lr_tol{tol}"]
    rl = np.array(g["ragged_lo"], np.int16)
    rh = np.array(g["ragged_hi"], np.int16)
    roff = np.concatenate([[0], np.cumsum(rh - rl + 1)]).astype(np.uint32)
    rS = np.concatenate([S[x, rl[x]:rh[x] + 1] for x in range(4)])
    assert orc.right_map(rS, 4, 1, 3, rl, rh, roff).ravel().tolist() == g["ragged_right"]


def test_sgm_lr_marks_invalid(orc):
    left, right, _ = synth.planes_pair(96, 32, seed=14)
    r = orc.sgm(left, right, 40)
    bad = r["disp_wta"] < 0
    assert bad.any() and (~bad).any()
    assert (r["disp_sub"][bad] == -1.0).all() and (r["var_meas"][bad] == 0).all()
    ok = ~bad
    assert np.array_equal(r["disp_wta"][ok], r["wta_raw"][ok])
    # the left border strip can never be matched (x - d < 0 for d >= 1 ...)
    assert (r["disp_wta"][:, 0][r["wta_raw"][:, 0] > 0] == -1).all()


# ---------------------------------------------------------------- windows
def test_windows_cases(orc):
    D = 128
    d = np.array([10.5, 10.49, 1.0, -1.0, 200.0, np.nan, 0.0, 127.0], np.float32)
    lo, hi, off = orc.windows(d, None, D, r_fixed=4)
    assert lo.tolist() == [7, 6, 0, 0, 0, 0, 0, 123]
    assert hi.tolist() == [15, 14, 5, 127, 127, 127, 4, 127]
    assert off.tolist() == list(np.concatenate([[0], np.cumsum(hi.astype(int) - lo + 1)]))
    # radius from the variance: ceil(3 sqrt(p)), clamped to [r_min, r_max]
    d = np.full(6, 50.0, np.float32)
    p = np.array([1.0, 1.0001, 0.0, 100.0, -1.0, np.inf], np.float32)
    lo, hi, _ = orc.windows(d, p, D, r_min=2, r_max=16)
    assert (hi - lo).tolist() == [6, 8, 4, 32, 127, 32]
    lo, hi, off = orc.windows(None, 30, 64)
    assert (lo == 0).all() and (hi == 63).all() and off[-1] == 30 * 64


# ---------------------------------------------------------------- warp
def _rot(yaw, pitch=0.0, roll=0.0):
    cy_, sy_ = np.cos(yaw), np.sin(yaw)
    cp, sp = np.cos(pitch), np.sin(pitch)
    cr, sr = np.cos(roll), np.sin(roll)
    Ry = np.array([[cy_, 0, sy_], [0, 1, 0], [-sy_, 0, cy_]])
    Rx = np.array([[1, 0, 0], [0, cp, -sp], [0, sp, cp]])
    Rz = np.array([[cr, -sr, 0], [sr, cr, 0], [0, 0, 1]])
    return Ry @ Rx @ Rz


CAM = dict(f=718.0, cx=40.5, cy=20.0, b=0.54)


def test_warp_identity(orc):
    r = np.random.default_rng(9)
    d = r.uniform(1.0, 100.0, size=(24, 40)).astype(np.float32)
    p = r.uniform(0.0, 5.0, size=(24, 40)).astype(np.float32)
    H = orc.warp_matrix(np.eye(3), np.zeros(3), **CAM)
    assert np.abs(H - np.eye(4)).max() < 1e-12
    assert np.array_equal(H.astype(np.float32), np.eye(4, dtype=np.float32))
    out = orc.warp(d, p, np.eye(3), np.zeros(3), q=0.5, **CAM)
    assert np.array_equal(out["winner"].ravel(), np.arange(24 * 40))
    assert np.array_equal(out["d_key_f32"], d)
    assert np.array_equal(out["d_pred"], d.astype(np.float64))
    assert np.array_equal(out["p_pred"], p.astype(np.float64) + 0.5)
    assert np.abs(out["d_pred"] - d).max() < 1e-9


def _reproject(x, y, d, R, t, f, cx, cy, b):
    Z = f * b / d
    X = (x - cx) * Z / f
    Y = (y - cy) * Z / f
    M = R @ np.stack([X, Y, Z]) + t[:, None]
    return f * M[0] / M[2] + cx, f * M[1] / M[2] + cy, f * b / M[2]


def test_warp_matrix_matches_euclidean_reprojection(orc):
    r = np.random.default_rng(10)
    for _ in range(10):
        R = _rot(*r.normal(0, 0.05, size=3))
        t = r.normal(0, 0.5, size=3)
        H = orc.warp_matrix(R, t, **CAM)
        x, y, d = r.uniform(0, 80, 50), r.uniform(0, 40, 50), r.uniform(2, 100, 50)
        om = H @ np.stack([x, y, d, np.ones_like(x)])
        xe, ye, de = _reproject(x, y, d, R, t, **CAM)
        assert np.allclose(om[0] / om[3], xe, rtol=0, atol=1e-9)
        assert np.allclose(om[1] / om[3], ye, rtol=0, atol=1e-9)
        assert np.allclose(om[2] / om[3], de, rtol=1e-12)


def test_warp_values_match_reprojection(orc):
    r = np.random.default_rng(11)
    h, w = 30, 80
    d = r.uniform(5, 60, size=(h, w)).astype(np.float32)
    p = r.uniform(0.1, 3, size=(h, w)).astype(np.float32)
    R, t = _rot(0.01, 0.002, -0.003), np.array([0.05, -0.02, -1.0])
    out = orc.warp(d, p, R, t, q=0.5, **CAM)
    win = out["winner"].ravel()
    ok = win >= 0
    assert ok.mean() > 0.5
    sx, sy = (win[ok] % w).astype(float), (win[ok] // w).astype(float)
    sd = d.ravel()[win[ok]].astype(float)
    xe, ye, de = _reproject(sx, sy, sd, R, t, **CAM)
    assert np.allclose(out["d_pred"].ravel()[ok], de, rtol=1e-12)
    tx, ty = np.nonzero(ok.reshape(h, w))[1], np.nonzero(ok.reshape(h, w))[0]
    assert (np.abs(xe - tx) <= 0.5 + 1e-4).all() and (np.abs(ye - ty) <= 0.5 + 1e-4).all()
    phi = de / sd
    assert np.allclose(out["p_pred"].ravel()[ok], phi * phi * p.ravel()[win[ok]] + 0.5,
                       rtol=1e-12)
    # the float32 values the z-buffer compared agree with the double ones
    assert np.abs(out["d_key_f32"].ravel()[ok] - out["d_pred"].ravel()[ok]).max() < 1e-4


def test_warp_forward_translation_closed_form(orc):
    h, w = 20, 60
    cam = dict(f=500.0, cx=29.5, cy=9.5, b=0.5)
    d = np.full((h, w), 10.0, np.float32)
    p = np.full((h, w), 2.0, np.float32)
    tau = 1.0
    out = orc.warp(d, p, np.eye(3), np.array([0, 0, -tau]), q=0.25, **cam)
    fb = cam["f"] * cam["b"]
    dn = 10.0 * fb / (fb - tau * 10.0)        # Z' = Z - tau
    v = out["winner"] >= 0
    assert np.allclose(out["d_pred"][v], dn, rtol=1e-12)
    assert np.allclose(out["p_pred"][v], (dn / 10.0) ** 2 * 2.0 + 0.25, rtol=1e-12)
    # the image expands about the principal point: holes appear (zoom effect)
    assert (~v).sum() > 0


def test_warp_zbuffer_keeps_nearest(orc):
    # Lateral motion t = (b,0,0) moves a pixel by x' = x + d; sources (2,0)
    # with d=3 and (4,0) with d=1 both land on x'=5: the larger d wins.
    cam = dict(f=100.0, cx=0.0, cy=0.0, b=0.5)
    d = np.full((1, 12), -1.0, np.float32)
    p = np.ones((1, 12), np.float32)
    d[0, 2], d[0, 4] = 3.0, 1.0
    p[0, 4] = 0.1
    out = orc.warp(d, p, np.eye(3), np.array([0.5, 0, 0]), q=0.5, **cam)
    assert out["winner"][0, 5] == 2 and out["d_pred"][0, 5] == pytest.approx(3.0)
    assert (out["winner"][0, [0, 1, 2, 3, 4, 6, 7, 8, 9, 10, 11]] == -1).all()
    assert (out["d_pred"][out["winner"] < 0] == -1.0).all()
    # Equal predicted disparity: moving back by tau contracts the image about
    # the principal point, x' = x fb/(fb + tau d); with fb = 100, d = 2 and
    # tau = 61.1 the factor is 0.45, so x=2 -> 0.9 and x=3 -> 1.35 both land on
    # pixel 1 with the same d'.  The paper is silent on such ties; the source
    # with the smaller pixel index is kept, whatever the variances.
    cam2 = dict(f=100.0, cx=0.0, cy=0.0, b=1.0)
    t = np.array([0.0, 0, 100.0 / 0.45 / 2 - 50.0])
    for p2, p3 in ((4.0, 1.0), (1.0, 4.0)):
        d = np.array([[-1, -1, 2.0, 2.0, -1, -1]], np.float32)
        p = np.array([[1, 1, p2, p3, 1, 1]], np.float32)
        out = orc.warp(d, p, np.eye(3), t, q=0.5, **cam2)
        assert out["winner"][0, 1] == 2
        assert out["d_pred"][0, 1] == pytest.approx(0.9)
        assert out["p_pred"][0, 1] == pytest.approx(0.45 ** 2 * p2 + 0.5)
        assert (out["winner"][0, [0, 2, 3, 4, 5]] == -1).all()


def test_warp_drops_invalid_and_outside(orc):
    cam = dict(f=100.0, cx=0.0, cy=0.0, b=0.5)
    d = np.array([[0.0, -1.0, np.nan, 5.0, 5.0]], np.float32)
    p = np.ones((1, 5), np.float32)
    out = orc.warp(d, p, np.eye(3), np.array([0.5, 0, 0]), q=0.5, **cam)
    # x' = x + d: 3 -> 8 and 4 -> 9 leave the 5-wide image
    assert (out["winner"] == -1).all()


# ---------------------------------------------------------------- Kalman
def test_kalman_closed_form_and_limits(orc):
    r = np.random.default_rng(12)
    n = 1000
    dp = r.uniform(0, 100, n).astype(np.float32)
    pp = r.uniform(0.01, 10, n).astype(np.float32)
    z = (dp + r.normal(0, 2, n)).clip(0).astype(np.float32)
    rr = r.integers(0, 20, n).astype(np.float32)
    d, p = orc.kalman(dp, pp, z, rr)
    D, P, Z, RR = (a.astype(np.float64) for a in (dp, pp, z, rr))
    assert np.allclose(d, (D * RR + Z * P) / (P + RR), rtol=1e-12, atol=1e-12)
    assert np.allclose(p, P * RR / (P + RR), rtol=1e-12, atol=1e-12)
    d0, p0 = orc.kalman(dp, pp, z, np.zeros(n, np.float32))
    assert np.array_equal(d0, Z) and np.all(p0 == 0)
    dm, pm = orc.kalman(dp, pp, z, pp)
    assert np.allclose(dm, (D + Z) / 2, rtol=1e-12) and np.allclose(pm, P / 2, rtol=1e-12)


def test_kalman_validity_table(orc):
    dp = np.array([5, -1, 5, -1, 5], np.float32)
    pp = np.array([1, 1, 1, 1, 0], np.float32)
    z = np.array([-1, 7, -1, -1, 6], np.float32)
    r = np.array([2, 3, 2, 2, 2], np.float32)
    d, p = orc.kalman(dp, pp, z, r)
    assert d.tolist() == [-1, 7, -1, -1, 6] and p.tolist() == [0, 3, 0, 0, 2]
    d, p = orc.kalman(dp, pp, z, r, keep_unmeasured=1)
    assert d.tolist() == [5, 7, 5, -1, 6] and p.tolist() == [1, 3, 1, 0, 2]


# ---------------------------------------------------------------- refinement
def test_refine_golden(orc):
    g = load("refine_hand.txt")
    d, p = orc.refine(np.array(g["d_in"], np.float32), np.array(g["p_in"], np.float32),
                      edge_tol=-1.0, fill_tol=1.0)
    assert np.array_equal(d, np.array(g["d_out"], np.float32))
    assert np.array_equal(p, np.array(g["p_out"], np.float32))
    v = np.array(g["v_in"], np.float32)
    d, p = orc.refine(v, np.ones_like(v), fill_tol=1.0)
    assert np.array_equal(d, np.array(g["v_out"], np.float32))
    assert np.array_equal(p[v < 0] > 0, np.array(g["v_out"])[v < 0] > 0)
    e = np.array(g["e_in"], np.float32)
    d, _ = orc.refine(e, np.ones_like(e), edge_tol=2.0, fill_tol=0.0)
    assert np.array_equal(d, np.array(g["e_out"], np.float32))


def test_refine_properties(orc):
    r = np.random.default_rng(13)
    d = r.uniform(0, 60, size=(30, 50)).astype(np.float32)
    p = r.uniform(0.1, 3, size=(30, 50)).astype(np.float32)
    # no holes, no edge test: identity
    od, op = orc.refine(d, p, edge_tol=-1.0, fill_tol=1.0)
    assert np.array_equal(od, d) and np.array_equal(op, p)
    # a smooth ramp with every other column missing is filled exactly
    ramp = np.tile(np.arange(50, dtype=np.float32) * 0.25, (30, 1))
    holes = ramp.copy()
    holes[:, 1::2] = -1
    od, _ = orc.refine(holes, np.ones_like(holes), fill_tol=1.0)
    assert np.array_equal(od[:, :-1], ramp[:, :-1])   # the last column has no right neighbour
    # dissimilar neighbours never fill: gaps between 10 and 20 stay
    d2 = np.tile(np.array([10, -1, 20, -1, 10], np.float32), (5, 1))
    od, _ = orc.refine(d2, np.ones_like(d2), fill_tol=1.0)
    assert (od[:, [1, 3]] == -1).all()
    # edge rejection only removes pixels, and only near jumps larger than the tolerance
    step = np.ones((8, 8), np.float32) * 5
    step[:, 4:] = 9
    od, _ = orc.refine(step, np.ones_like(step), edge_tol=3.0, fill_tol=0.0)
    assert (od[:, [3, 4]] == -1).all() and (od[:, [0, 1, 2, 5, 6, 7]] >= 0).all()
    od, _ = orc.refine(step, np.ones_like(step), edge_tol=4.0, fill_tol=0.0)
    assert np.array_equal(od, step)


# ------------------------------------------------------------- SAD check
def test_sad_check_window_and_threshold_by_hand(orc):
    """Left all 10, right all 13, radius 1, d = 0: every 3x3 sum is 9 * 3 = 27;
    the check rejects strictly above sad_max."""
    left = np.full((3, 5), 10, np.uint8)
    right = np.full((3, 5), 13, np.uint8)
    d = np.zeros((3, 5), np.int16)
    wta, sub, var = orc.sad_check(left, right, d, 1, 27, np.zeros((3, 5)), np.ones((3, 5)))
    assert (wta == 0).all() and (var == 1).all()
    wta, sub, var = orc.sad_check(left, right, d, 1, 26, np.zeros((3, 5)), np.ones((3, 5)))
    assert (wta == -1).all() and (sub == -1).all() and (var == 0).all()


def test_sad_check_clamps_coordinates_into_the_image(orc):
    """Right column 0 holds 50, the rest 0; left all 50.  At x = 0 with d = 2
    every right tap falls left of the image and is clamped to column 0, so
    the sum is 0 (zero padding would give 50 per tap)."""
    left = np.full((4, 4), 50, np.uint8)
    right = np.zeros((4, 4), np.uint8)
    right[:, 0] = 50
    d = np.full((4, 4), -1, np.int16)
    d[1, 0] = 2
    wta, _, _ = orc.sad_check(left, right, d, 1, 0)
    assert wta[1, 0] == 2
    d2 = d.copy()
    d2[1, 0], d2[2, 3] = -1, 1          # x=3, d=1: taps x+i-1 in 1..3, right there is 0
    wta, _, _ = orc.sad_check(left, right, d2, 1, 450)
    assert wta[2, 3] == 1               # 9 taps * |50 - 0| = 450, not above 450: kept
    wta, _, _ = orc.sad_check(left, right, d2, 1, 449)
    assert wta[2, 3] == -1              # above 449: rejected
    assert (wta[d2 < 0] == -1).all()    # pixels without a disparity are left alone


def test_sad_check_exact_shift_keeps_interior(orc):
    left, right = synth.shifted_pair(60, 20, 7, seed=21)
    d = np.full((20, 60), 7, np.int16)
    wta, _, _ = orc.sad_check(left, right, d, 2, 0)
    assert (wta[2:-2, 9:-2] == 7).all()      # x - d - r >= 0 and inside the rows


# ------------------------------------------- left-right check of a prediction
def test_right_camera_motion_moves_points_like_the_left_one(orc):
    """M_R = M_L - (b,0,0): moving points with (R, t) in the left frame equals
    moving them with (R, t_R) in the right frame."""
    g = np.random.default_rng(3)
    R = np.eye(3) + g.normal(0, 0.1, (3, 3))   # the relation is linear: any matrix will do
    t = g.normal(0, 1, 3)
    b = 0.54
    tr = orc.right_motion(R, t, b)
    M = g.normal(0, 5, (3, 20))
    bv = np.array([[b], [0.0], [0.0]])
    lhs = (R @ M + t[:, None]) - bv
    rhs = R @ (M - bv) + tr[:, None]
    assert np.allclose(lhs, rhs, atol=1e-12)


def test_lr_check_prediction_by_hand(orc):
    #   x:        0     1     2     3     4     5
    d = np.array([[0.4, 2.6, 1.0, -1.0, 3.49, 5.0]], np.float32)
    p = np.ones_like(d)
    dr = np.array([[0.0, 9.0, 1.9, -1.0, 7.0, 6.0]], np.float32)
    # x=0: xr = 0 - 0 = 0, |0 - 0.4| <= 1 keep; x=1: xr = 1 - 3 < 0 reject;
    # x=2: xr = 1, |9 - 1| > 1 reject; x=3: no prediction (left alone);
    # x=4: xr = 4 - 3 = 1, |9 - 3.49| > 1 reject; x=5: xr = 0, |0 - 5| reject.
    out_d, out_p = orc.lr_check_prediction(d, p, dr, 1.0)
    assert out_d.tolist() == [[np.float32(0.4), -1.0, -1.0, -1.0, -1.0, -1.0]]
    assert out_p.tolist() == [[1.0, 0.0, 0.0, 1.0, 0.0, 0.0]]
    dr2 = dr.copy()
    dr2[0, 1] = 1.9                          # x=2 (xr=1): |1.9 - 1| <= 1 now kept
    out_d, _ = orc.lr_check_prediction(d, p, dr2, 1.0)
    assert out_d[0, 2] == np.float32(1.0)
    out_d, _ = orc.lr_check_prediction(d, p, dr2, 0.8)
    assert out_d[0, 2] == -1.0               # tolerance is a float32 <=


def test_warped_maps_of_a_plane_stay_consistent(orc):
    """A fronto-parallel plane at Z: left and right maps are the constant
    fb/Z; after moving forward both warped predictions are the same constant
    where defined, so the check keeps every left pixel whose partner is in
    the image."""
    w, h, f, b = 90, 30, 60.0, 0.5
    cx, cy = (w - 1) / 2, (h - 1) / 2
    d0 = f * b / 10.0
    dl = np.full((h, w), d0, np.float32)
    dr = np.full((h, w), d0, np.float32)
    dr[:, w - int(np.floor(d0 + 0.5)):] = -1.0            # right pixels whose left partner is outside
    R, t = np.eye(3), np.array([0.0, 0.0, -1.0])
    wl = orc.warp(dl, np.ones_like(dl), R, t, f, cx, cy, b, 0.5)
    wr = orc.warp(dr, np.ones_like(dr), R, orc.right_motion(R, t, b), f, cx, cy, b, 0.5)
    d1 = f * b / 9.0
    okl = wl["d_pred"] >= 0
    assert np.allclose(wl["d_pred"][okl], d1, atol=1e-9)
    assert np.allclose(wr["d_pred"][wr["d_pred"] >= 0], d1, atol=1e-9)
    out_d, _ = orc.lr_check_prediction(wl["d_pred"].astype(np.float32), wl["p_pred"].astype(np.float32),
                                       wr["d_pred"].astype(np.float32), 1.0)
    kept = out_d >= 0
    xs = np.arange(w)[None, :].repeat(h, 0)
    inner = okl & (xs - np.floor(d1 + 0.5) >= 0)
    inner &= np.take_along_axis(wr["d_pred"] >= 0, np.clip(xs - int(np.floor(d1 + 0.5)), 0, w - 1), 1)
    assert np.array_equal(kept, inner)
    # the zoom leaves one-pixel holes in both maps; filled first (the order of
    # Fig. 4), the interior is kept entirely
    fl, pl = orc.refine(wl["d_pred"].astype(np.float32), wl["p_pred"].astype(np.float32), -1.0, 1.0)
    fr, _ = orc.refine(wr["d_pred"].astype(np.float32), wr["p_pred"].astype(np.float32), -1.0, 1.0)
    out_d, _ = orc.lr_check_prediction(fl, pl, fr, 1.0)
    assert (out_d[3:-3, 6:-6] >= 0).all()
