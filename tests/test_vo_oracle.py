"""Pins of the ego-motion oracle (oracle/vo.py) against facts outside it:
library routines for the SE(3) exponential, finite differences for the
Jacobian, the renderer's exact camera motion, and closed forms of the
pyramid's camera and a motionless pair."""
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

from oracle import vo
from paper_1708_06301_amd import synth


def _pose_error(R, t, Rg, tg):
    dR = R @ Rg.T
    ang = np.degrees(np.arccos(np.clip((np.trace(dR) - 1.0) / 2.0, -1.0, 1.0)))
    return float(np.linalg.norm(t - tg)), float(ang)


@pytest.mark.parametrize("xi", [[0.3, -0.2, 0.5, 0.2, -0.4, 0.1], [1.0, 0.0, 0.0, 0.0, 0.0, 0.0],
                                [0.0, 0.0, 0.0, 1e-10, 2e-10, -1e-10], [0.1, 0.2, 0.3, 2.5, -1.0, 0.5]])
def test_se3_exp_equals_the_matrix_exponential(xi):
    """exp of the twist (rho, phi) is the matrix exponential of [[phi]x rho; 0 0]
    (scipy's expm), and its rotation is Rodrigues' (scipy's rotation vector)."""
    R, t = vo.se3_exp(xi)
    T = np.zeros((4, 4))
    T[:3, :3] = vo.hat(xi[3:])
    T[:3, 3] = xi[:3]
    E = expm(T)
    assert np.allclose(R, E[:3, :3], atol=1e-12)
    assert np.allclose(t, E[:3, 3], atol=1e-12)
    assert np.allclose(R, Rotation.from_rotvec(xi[3:]).as_matrix(), atol=1e-12)


def test_jacobian_matches_finite_differences():
    """The analytic Jacobian of the residual w.r.t. the left-multiplied twist
    against central differences of the oracle's own residual, on a smooth
    image pair and a sloped disparity plane (a sign or an index mistake
    flips or scrambles a column)."""
    h, w = 96, 160
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)

    def img(sx, sy):
        return (128 + 50 * np.sin(0.11 * (xx + sx)) * np.cos(0.09 * (yy + sy)) +
                30 * np.sin(0.05 * (xx + sx) + 0.07 * (yy + sy)))

    I0, I1 = img(0, 0).astype(np.float32), img(1.5, 0.7).astype(np.float32)
    D = (15.0 + 10.0 * yy / h).astype(np.float32)
    prm = vo.VOParams(levels=1, iters=(1,))
    L = vo.Levels(I0, I1, D, 200.0, 79.5, 47.5, 0.5, prm)
    args = (L.ref[0], L.disp[0], L.cur[0], *L.grad[0], L.cams[0])
    R, t = vo.se3_exp([0.01, -0.02, 0.03, 0.001, -0.002, 0.0015])
    t = t + np.array([0.02, -0.01, 0.05])
    ok, _, J, _ = vo.warp_terms(*args, R, t, prm, 0)
    eps = 1e-5
    for i in range(6):
        e = np.zeros(6)
        e[i] = eps
        Rp, tp = vo.se3_exp(e)
        Rm, tm = vo.se3_exp(-e)
        okp, rp, _, _ = vo.warp_terms(*args, Rp @ R, Rp @ t + tp, prm, 0)
        okm, rm, _, _ = vo.warp_terms(*args, Rm @ R, Rm @ t + tm, prm, 0)
        m = ok & okp & okm
        fd = (rp - rm)[m] / (2 * eps)
        a = J[m, i]
        assert m.sum() > 10000
        assert np.corrcoef(a, fd)[0, 1] > 0.999, i
        assert np.linalg.norm(a - fd) / np.linalg.norm(fd) < 0.06, i


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("noise", [False, True])
def test_recovers_the_renderers_motion(k, noise):
    """With the true disparity of frame k-1, the estimate from the identity
    recovers the renderer's exact motion (1 m forward with a small yaw)."""
    seq = synth.street_sequence(480, 144, 4, seed=synth.seed_for(1))
    cam = seq.cam
    L0, _, gt0 = seq.frame(k - 1, noise=noise)
    L1, _, _ = seq.frame(k, noise=noise)
    Rg, tg = seq.motion(k)
    R, t = vo.estimate_motion(L0, L1, gt0.astype(np.float32), cam.f, cam.cx, cam.cy, cam.baseline,
                              vo.VOParams(levels=4, iters=(2, 4, 8, 10)))
    et, er = _pose_error(R, t, Rg, tg)
    assert et < 0.005 and er < 0.02, (et, er)


def test_motionless_pair_stays_at_identity():
    seq = synth.street_sequence(480, 144, 2, seed=synth.seed_for(1))
    cam = seq.cam
    L0, _, gt0 = seq.frame(0, noise=False)
    R, t = vo.estimate_motion(L0, L0, gt0.astype(np.float32), cam.f, cam.cx, cam.cy, cam.baseline,
                              vo.VOParams(levels=4, iters=(2, 4, 8, 10)))
    et, er = _pose_error(R, t, np.eye(3), np.zeros(3))
    assert et < 1e-4 and er < 1e-3, (et, er)


def test_level_camera_keeps_points_on_their_pixels():
    """A 3-D point's projection at level l is (x0 + 0.5) / 2^l - 0.5 for its
    level-0 projection x0 (level-l pixel x averages level-0 pixels
    2^l x .. 2^l x + 2^l - 1), and Z = f_l b / d_l holds with d_l = d / 2^l."""
    f, cx, cy, b = 718.0, 620.5, 187.0, 0.54
    P = np.array([1.3, -0.4, 9.0])
    x0, y0 = f * P[0] / P[2] + cx, f * P[1] / P[2] + cy
    d0 = f * b / P[2]
    for l in range(5):
        fl, cxl, cyl, fbl = (float(v) for v in vo.level_camera(f, cx, cy, b, l))
        s = 2.0 ** l
        assert np.isclose(fl * P[0] / P[2] + cxl, (x0 + 0.5) / s - 0.5, atol=1e-4)
        assert np.isclose(fl * P[1] / P[2] + cyl, (y0 + 0.5) / s - 0.5, atol=1e-4)
        assert np.isclose(fbl / (d0 / s), P[2], rtol=1e-6)


def test_pyramids_by_hand():
    I = np.arange(32, dtype=np.uint8).reshape(4, 8)
    p = vo.image_pyramid(I, 3)
    assert p[1].shape == (2, 4) and p[2].shape == (1, 2)
    assert p[1][0, 0] == (0 + 1 + 8 + 9) / 4.0 and p[1][1, 3] == (22 + 23 + 30 + 31) / 4.0
    gx, gy = vo.gradients(p[0])
    assert gx[1, 1] == 1.0 and gy[1, 1] == 8.0 and gx[0, 0] == 0.0 and gy[3, 5] == 0.0
    d = np.array([[4.0, 9.0, -1.0, 3.0], [1.0, 1.0, 1.0, 1.0]], np.float32)
    q = vo.disparity_pyramid(d, 2)[1]
    assert q.tolist() == [[2.0, -1.0]]


def test_normal_equations_are_symmetric_and_positive():
    seq = synth.street_sequence(480, 144, 2, seed=synth.seed_for(1))
    cam = seq.cam
    L0, _, gt0 = seq.frame(0, noise=True)
    L1, _, _ = seq.frame(1, noise=True)
    L = vo.Levels(L0, L1, gt0.astype(np.float32), cam.f, cam.cx, cam.cy, cam.baseline, vo.VOParams(levels=3))
    H, g, cost, n = L.normal(1, np.eye(3), np.zeros(3))
    assert n > 1000 and cost > 0
    assert np.allclose(H, H.T)
    assert np.linalg.eigvalsh(H).min() > 0
