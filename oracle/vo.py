"""Oracle of the ego-motion front end: direct stereo visual odometry.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product library
never does, and it shares no code with the HIP path.

The paper takes the ego-motion T between consecutive stereo frames from a
visual odometry algorithm it cites and does not describe (Sec. 1, Sec. 2.1).
This front end is the project's own: it estimates the motion that the warp of
Sec. 2.2 consumes (M_k = R M_{k-1} + t, Eq. 1-4) by aligning the previous
left image to the current one through the previous disparity map, i.e. it
minimises the photometric error

    E(R, t) = sum_p rho( I_k(pi(R P(p) + t)) - I_{k-1}(p) ),

where P(p) is pixel p of frame k-1 lifted to 3-D with its disparity
(Z = f b / d, the relation of Eq. 1) and pi the pinhole projection; rho is
Huber's function.  Gauss-Newton on a pyramid, coarse to fine, with a fixed
number of iterations per level.  The update is left-multiplicative,
T <- exp(xi) T, with xi = (rho, phi) (translation part, rotation part).

Precision: the lift, the motion and the projection, which decide the pixel
an image is sampled at and whether it lies inside the image, are evaluated
in float32 in a fixed operation order (the GPU path evaluates the same
expressions in float32); everything after them is float64 here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

f32 = np.float32


@dataclass
class VOParams:
    levels: int = 4
    # Gauss-Newton iterations per level, finest first (level 0 = full size)
    iters: tuple = (2, 4, 6, 6)
    huber: float = 8.0        # intensity units
    min_disp: float = 1.0     # pixels at level 0


# ------------------------------------------------------------------ SE(3)
def hat(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def se3_exp(xi):
    """exp of the twist xi = (rho, phi): rotation by Rodrigues' formula,
    translation V(phi) rho with V = I + (1-cos a)/a^2 [phi] + (a - sin a)/a^3 [phi]^2."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    a = float(np.linalg.norm(phi))
    K = hat(phi)
    K2 = K @ K
    if a < 1e-8:
        A, B, C = 1.0 - a * a / 6.0, 0.5 - a * a / 24.0, 1.0 / 6.0 - a * a / 120.0
    else:
        A, B, C = np.sin(a) / a, (1.0 - np.cos(a)) / (a * a), (a - np.sin(a)) / (a ** 3)
    R = np.eye(3) + A * K + B * K2
    V = np.eye(3) + B * K + C * K2
    return R, V @ rho


# --------------------------------------------------------------- pyramids
def image_pyramid(img_u8, levels):
    """float32 images; level l is the 2x2 mean of level l-1, ((a+b)+(c+d))*0.25."""
    out = [np.asarray(img_u8, np.float32)]
    for _ in range(1, levels):
        I = out[-1]
        h, w = I.shape[0] // 2, I.shape[1] // 2
        a = I[0:2 * h:2, 0:2 * w:2]
        b = I[0:2 * h:2, 1:2 * w:2]
        c = I[1:2 * h:2, 0:2 * w:2]
        d = I[1:2 * h:2, 1:2 * w:2]
        out.append(((a + b) + (c + d)) * f32(0.25))
    return out


def gradients(I):
    """Central differences (I(x+1) - I(x-1)) * 0.5 in float32, zero on the border."""
    gx = np.zeros_like(I)
    gy = np.zeros_like(I)
    gx[:, 1:-1] = (I[:, 2:] - I[:, :-2]) * f32(0.5)
    gy[1:-1, :] = (I[2:, :] - I[:-2, :]) * f32(0.5)
    return gx, gy


def disparity_pyramid(d, levels):
    """Level l samples level l-1 at (2x, 2y) and halves it; invalid (<= 0) stays -1."""
    out = [np.asarray(d, np.float32)]
    for _ in range(1, levels):
        D = out[-1]
        h, w = D.shape[0] // 2, D.shape[1] // 2
        s = D[0:2 * h:2, 0:2 * w:2]
        out.append(np.where(s > 0, s * f32(0.5), f32(-1.0)).astype(np.float32))
    return out


def level_camera(f, cx, cy, baseline, l):
    """Camera of level l (pixel x of level l covers level-0 pixels 2^l x .. 2^l x + 2^l - 1):
    f/2^l, (c + 0.5)/2^l - 0.5; and f_l * b, the numerator of Z = f b / d."""
    s = 2.0 ** l
    fl = f / s
    return f32(fl), f32((cx + 0.5) / s - 0.5), f32((cy + 0.5) / s - 0.5), f32(fl * baseline)


# ------------------------------------------------------- one level's terms
def warp_terms(Iref, D, Icur, Gx, Gy, cam, R, t, prm: VOParams, l):
    """Per reference pixel: mask of pixels that enter the sum, residual r,
    Jacobian J (n x 6, w.r.t. xi = (rho, phi)) and Huber weight w (float64),
    for the motion (R, t) at pyramid level l."""
    fl, cxl, cyl, fbl = cam
    h, w = Iref.shape
    md = f32(prm.min_disp / 2.0 ** l)
    vv, uu = np.meshgrid(np.arange(h, dtype=np.float32), np.arange(w, dtype=np.float32), indexing="ij")
    d = D
    ok = d >= md
    dd = np.where(ok, d, f32(1.0))
    R32 = np.asarray(R, np.float64).astype(np.float32)
    t32 = np.asarray(t, np.float64).astype(np.float32)
    # float32, in this order (the lift of Eq. 1, the motion, the projection)
    Z = fbl / dd
    X = ((uu - cxl) * Z) / fl
    Y = ((vv - cyl) * Z) / fl
    Xp = ((R32[0, 0] * X + R32[0, 1] * Y) + R32[0, 2] * Z) + t32[0]
    Yp = ((R32[1, 0] * X + R32[1, 1] * Y) + R32[1, 2] * Z) + t32[1]
    Zp = ((R32[2, 0] * X + R32[2, 1] * Y) + R32[2, 2] * Z) + t32[2]
    zs = np.where(Zp > 0, Zp, f32(1.0))
    up = (fl * Xp) / zs + cxl
    vp = (fl * Yp) / zs + cyl
    ok &= (Zp > 0) & (up >= f32(1.0)) & (up < f32(w - 2)) & (vp >= f32(1.0)) & (vp < f32(h - 2))
    x0 = np.floor(np.where(ok, up, f32(1.0))).astype(np.int64)
    y0 = np.floor(np.where(ok, vp, f32(1.0))).astype(np.int64)
    fx = np.where(ok, up - x0.astype(np.float32), f32(0.0)).astype(np.float64)
    fy = np.where(ok, vp - y0.astype(np.float32), f32(0.0)).astype(np.float64)

    def bilinear(img):
        I = img.astype(np.float64)
        return ((1 - fy) * ((1 - fx) * I[y0, x0] + fx * I[y0, x0 + 1]) +
                fy * ((1 - fx) * I[y0 + 1, x0] + fx * I[y0 + 1, x0 + 1]))

    r = bilinear(Icur) - Iref.astype(np.float64)
    gx, gy = bilinear(Gx), bilinear(Gy)
    X1, Y1, Z1 = Xp.astype(np.float64), Yp.astype(np.float64), zs.astype(np.float64)
    F = float(fl)
    ju = gx * F / Z1
    jv = gy * F / Z1
    jz = -(gx * F * X1 + gy * F * Y1) / (Z1 * Z1)
    # d(pi(P'))/d(xi) with dP'/d(xi) = [I | -[P']x]: rotation columns are P' x (ju, jv, jz)
    J = np.stack([ju, jv, jz, Y1 * jz - Z1 * jv, Z1 * ju - X1 * jz, X1 * jv - Y1 * ju], -1)
    a = np.abs(r)
    wgt = np.where(a <= prm.huber, 1.0, prm.huber / np.maximum(a, 1e-300))
    return ok, r, J, wgt


def normal_equations(Iref, D, Icur, Gx, Gy, cam, R, t, prm, l):
    """H = sum w J^T J, g = sum w J r, cost = sum w r^2 and the pixel count."""
    ok, r, J, wgt = warp_terms(Iref, D, Icur, Gx, Gy, cam, R, t, prm, l)
    Jm, rm, wm = J[ok], r[ok], wgt[ok]
    H = (Jm * wm[:, None]).T @ Jm
    g = (Jm * wm[:, None]).T @ rm
    return H, g, float(np.sum(wm * rm * rm)), int(ok.sum())


def gauss_newton_step(H, g, n):
    """xi = -(H + lambda I)^-1 g with lambda = 1e-9 trace(H)/6 (no update below 16 pixels)."""
    if n < 16:
        return np.zeros(6)
    lam = 1e-9 * np.trace(H) / 6.0
    return -np.linalg.solve(H + lam * np.eye(6), g)


class Levels:
    """Pyramids of one frame pair."""

    def __init__(self, prev_u8, cur_u8, prev_disp, f, cx, cy, baseline, prm: VOParams):
        self.prm = prm
        self.ref = image_pyramid(prev_u8, prm.levels)
        self.cur = image_pyramid(cur_u8, prm.levels)
        self.grad = [gradients(I) for I in self.cur]
        self.disp = disparity_pyramid(prev_disp, prm.levels)
        self.cams = [level_camera(f, cx, cy, baseline, l) for l in range(prm.levels)]

    def normal(self, l, R, t):
        return normal_equations(self.ref[l], self.disp[l], self.cur[l], *self.grad[l], self.cams[l],
                                R, t, self.prm, l)


def estimate_motion(prev_u8, cur_u8, prev_disp, f, cx, cy, baseline, prm: VOParams = VOParams(),
                    R0=None, t0=None):
    """(R, t) with M_k = R M_{k-1} + t, from the previous left image and
    disparity map and the current left image, starting at (R0, t0)."""
    L = Levels(prev_u8, cur_u8, prev_disp, f, cx, cy, baseline, prm)
    R = np.eye(3) if R0 is None else np.asarray(R0, np.float64).copy()
    t = np.zeros(3) if t0 is None else np.asarray(t0, np.float64).copy()
    for l in range(prm.levels - 1, -1, -1):
        for _ in range(prm.iters[l]):
            H, g, _, n = L.normal(l, R, t)
            Rd, td = se3_exp(gauss_newton_step(H, g, n))
            R, t = Rd @ R, Rd @ t + td
    return R, t
