"""Seeded synthetic stereo inputs.

This module generates inputs only: textures, stereo pairs with a known
disparity field, and ray-cast image sequences of a static street-like scene
(ground plane, boxes, distant backdrop) seen by a stereo rig that drives
forward with a small random yaw per frame.  It holds none of the matcher's,
warp's or filter's arithmetic and is shared by the tests, the benchmark and
the smoke check, which feed the same arrays to the GPU library and to the
CPU oracle.

Everything is a pure function of an integer seed.  Seeds are mixed with
splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", 2014); coherent texture is Perlin's improved noise (Perlin,
"Improving noise", SIGGRAPH 2002), evaluated in float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 1708063
_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One splitmix64 output for state x (the state advance included)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def seed_for(config: int, index: int = 0, salt: int = 0) -> int:
    return splitmix64(splitmix64(BASE_SEED + config) ^ (index * 0x100000001B3 + salt))


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# Perlin improved noise
# --------------------------------------------------------------------------
class Perlin:
    """Improved Perlin noise in 2-D and 3-D with a seeded permutation."""

    def __init__(self, seed: int):
        perm = rng(seed).permutation(256).astype(np.int64)
        self.p = np.concatenate([perm, perm])

    @staticmethod
    def _fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    @staticmethod
    def _grad3(h, x, y, z):
        h = h & 15
        u = np.where(h < 8, x, y)
        v = np.where(h < 4, y, np.where((h == 12) | (h == 14), x, z))
        return np.where(h & 1, -u, u) + np.where(h & 2, -v, v)

    def noise3(self, x, y, z):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        z = np.asarray(z, np.float64)
        fx, fy, fz = np.floor(x), np.floor(y), np.floor(z)
        X = fx.astype(np.int64) & 255
        Y = fy.astype(np.int64) & 255
        Z = fz.astype(np.int64) & 255
        x, y, z = x - fx, y - fy, z - fz
        u, v, w = self._fade(x), self._fade(y), self._fade(z)
        p = self.p
        A = p[X] + Y
        AA, AB = p[A] + Z, p[A + 1] + Z
        B = p[X + 1] + Y
        BA, BB = p[B] + Z, p[B + 1] + Z
        g = self._grad3

        def lerp(t, a, b):
            return a + t * (b - a)

        return lerp(w,
                    lerp(v, lerp(u, g(p[AA], x, y, z), g(p[BA], x - 1, y, z)),
                         lerp(u, g(p[AB], x, y - 1, z), g(p[BB], x - 1, y - 1, z))),
                    lerp(v, lerp(u, g(p[AA + 1], x, y, z - 1), g(p[BA + 1], x - 1, y, z - 1)),
                         lerp(u, g(p[AB + 1], x, y - 1, z - 1), g(p[BB + 1], x - 1, y - 1, z - 1))))

    def noise2(self, x, y):
        return self.noise3(x, y, np.zeros_like(np.asarray(x, np.float64)) + 0.5)

    def fbm3(self, x, y, z, octaves=4):
        total = np.zeros(np.broadcast(np.asarray(x), np.asarray(y), np.asarray(z)).shape)
        amp, freq, norm = 1.0, 1.0, 0.0
        for _ in range(octaves):
            total = total + amp * self.noise3(x * freq, y * freq, z * freq)
            norm += amp
            amp *= 0.5
            freq *= 2.0
        return total / norm

    def fbm2(self, x, y, octaves=4):
        return self.fbm3(x, y, np.zeros_like(np.asarray(x, np.float64)) + 0.5, octaves)


def _to_u8(v):
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------
# Single pairs with a known disparity field
# --------------------------------------------------------------------------
def texture(w: int, h: int, seed: int, noise_sigma: float = 6.0, scale: float = 16.0):
    """uint8 texture: 128 + 180 fBm(x/scale, y/scale) + N(0, sigma^2)."""
    r = rng(seed)
    pn = Perlin(int(r.integers(0, 2**62)))
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    v = 128.0 + 180.0 * pn.fbm2(xx / scale, yy / scale)
    if noise_sigma > 0:
        v = v + r.normal(0.0, noise_sigma, size=v.shape)
    return _to_u8(v)


def plane_field(w: int, h: int, integer: bool = False):
    """Piecewise-planar disparity field in right-image coordinates: a
    slanted background plus two rectangles, disparities within 0..60."""
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    d = 6.0 + 18.0 * yy / max(h - 1, 1)
    ax0, ax1, ay0, ay1 = int(0.20 * w), int(0.45 * w), int(0.20 * h), int(0.70 * h)
    bx0, bx1, by0, by1 = int(0.60 * w), int(0.85 * w), int(0.35 * h), int(0.90 * h)
    a = (yy >= ay0) & (yy < ay1) & (xx >= ax0) & (xx < ax1)
    d = np.where(a, 30.0 + 0.05 * (xx - ax0), d)
    b = (yy >= by0) & (yy < by1) & (xx >= bx0) & (xx < bx1)
    d = np.where(b, 54.0, d)
    if integer:
        d = np.floor(d + 0.5)
    return d


def pair_from_field(left: np.ndarray, disp_right: np.ndarray, seed: int):
    """right(x', y) = left(x' + d(x', y), y), linearly interpolated; samples
    beyond the left image's right edge are fresh noise."""
    h, w = left.shape
    r = rng(seed)
    fresh = r.integers(0, 256, size=(h, w + 300)).astype(np.float64)
    ext = np.concatenate([left.astype(np.float64), fresh[:, : 300]], axis=1)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    xs = xx + disp_right
    x0 = np.floor(xs).astype(np.int64)
    fr = xs - x0
    x0 = np.clip(x0, 0, w + 299)
    x1 = np.clip(x0 + 1, 0, w + 299)
    yi = yy.astype(np.int64)
    v = (1.0 - fr) * ext[yi, x0] + fr * ext[yi, x1]
    return _to_u8(v)


def planes_pair(w: int = 320, h: int = 96, seed: int | None = None, integer: bool = False,
                noise_sigma: float = 6.0):
    """The 320x96 three-plane pair: (left, right, disparity in right coords)."""
    if seed is None:
        seed = seed_for(0)
    left = texture(w, h, splitmix64(seed ^ 1), noise_sigma=noise_sigma)
    d = plane_field(w, h, integer=integer)
    right = pair_from_field(left, d, splitmix64(seed ^ 2))
    return left, right, d


def shifted_pair(w: int, h: int, d0: int, seed: int):
    """Fronto-parallel integer plane: right(x', y) = left(x'+d0, y)."""
    left = texture(w, h, splitmix64(seed ^ 3), noise_sigma=20.0, scale=4.0)
    r = rng(splitmix64(seed ^ 4))
    right = np.empty_like(left)
    right[:, : w - d0] = left[:, d0:]
    right[:, w - d0:] = r.integers(0, 256, size=(h, d0), dtype=np.uint8)
    return left, right


# --------------------------------------------------------------------------
# Ray-cast sequences
# --------------------------------------------------------------------------
@dataclass
class Camera:
    w: int
    h: int
    f: float
    cx: float
    cy: float
    baseline: float

    @staticmethod
    def kitti_like(w: int = 1242, h: int = 375, f: float | None = None):
        f = 718.0 * w / 1242.0 if f is None else f
        return Camera(w, h, f, (w - 1) / 2.0, (h - 1) / 2.0, 0.54)


def _yaw(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


@dataclass
class Scene:
    """Static world: ground plane y = cam_height (camera axes: x right, y
    down, z forward), axis-aligned boxes standing on it and a backdrop
    sphere.  poses[k] = (Rwc, c): camera-to-world rotation and centre."""
    cam_height: float
    boxes: np.ndarray            # (n, 6): xmin, ymin, zmin, xmax, ymax, zmax
    backdrop_center: np.ndarray
    backdrop_radius: float
    poses: list = field(default_factory=list)
    tex_seed: int = 0
    noise_sigma: float = 2.0
    noise_seed: int = 0


def make_scene(seed: int, n_frames: int, step: float = 1.0, yaw_sigma_deg: float = 0.5,
               n_boxes: int = 12, cam_height: float = 1.65, noise_sigma: float = 2.0) -> Scene:
    r = rng(seed)
    Rwc = np.eye(3)
    c = np.zeros(3)
    poses = [(Rwc.copy(), c.copy())]
    for _ in range(1, n_frames):
        c = c + Rwc @ np.array([0.0, 0.0, step])
        Rwc = Rwc @ _yaw(np.deg2rad(r.normal(0.0, yaw_sigma_deg)))
        poses.append((Rwc.copy(), c.copy()))
    travel = step * max(n_frames - 1, 0)
    boxes = []
    for _ in range(n_boxes):
        s = r.uniform(8.0, 70.0 + travel)          # distance along the route
        k = min(int(s / max(step, 1e-9)), n_frames - 1) if travel > 0 else 0
        Rk, ck = poses[k]
        ahead = s - k * step
        lateral = r.uniform(3.0, 12.0) * (1.0 if r.random() < 0.5 else -1.0)
        centre = ck + Rk @ np.array([lateral, 0.0, ahead])
        sx, sy, sz = r.uniform(1.0, 4.0, size=3)
        boxes.append([centre[0] - sx / 2, cam_height - sy, centre[2] - sz / 2,
                      centre[0] + sx / 2, cam_height, centre[2] + sz / 2])
    mid = poses[len(poses) // 2][1]
    return Scene(cam_height=cam_height, boxes=np.array(boxes, np.float64),
                 backdrop_center=mid, backdrop_radius=150.0 + travel,
                 poses=poses, tex_seed=splitmix64(seed ^ 0xABCDEF),
                 noise_sigma=noise_sigma, noise_seed=splitmix64(seed ^ 0x123457))


def _perlin_torch(perm: np.ndarray, device):
    import torch
    return torch.as_tensor(np.concatenate([perm, perm]), dtype=torch.int64, device=device)


def _noise3_torch(p, x, y, z):
    """Improved Perlin noise on torch tensors (float64)."""
    import torch
    fx, fy, fz = torch.floor(x), torch.floor(y), torch.floor(z)
    X = fx.long() & 255
    Y = fy.long() & 255
    Z = fz.long() & 255
    x, y, z = x - fx, y - fy, z - fz

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def grad(hh, a, b, c):
        hh = hh & 15
        u = torch.where(hh < 8, a, b)
        v = torch.where(hh < 4, b, torch.where((hh == 12) | (hh == 14), a, c))
        return torch.where((hh & 1) != 0, -u, u) + torch.where((hh & 2) != 0, -v, v)

    def lerp(t, a, b):
        return a + t * (b - a)

    u, v, w = fade(x), fade(y), fade(z)
    A = p[X] + Y
    AA, AB = p[A] + Z, p[A + 1] + Z
    B = p[X + 1] + Y
    BA, BB = p[B] + Z, p[B + 1] + Z
    return lerp(w,
                lerp(v, lerp(u, grad(p[AA], x, y, z), grad(p[BA], x - 1, y, z)),
                     lerp(u, grad(p[AB], x, y - 1, z), grad(p[BB], x - 1, y - 1, z))),
                lerp(v, lerp(u, grad(p[AA + 1], x, y, z - 1), grad(p[BA + 1], x - 1, y, z - 1)),
                     lerp(u, grad(p[AB + 1], x, y - 1, z - 1), grad(p[BB + 1], x - 1, y - 1, z - 1))))


def _fbm3_torch(p, x, y, z, octaves=4):
    total = 0.0
    amp, freq, norm = 1.0, 1.0, 0.0
    for _ in range(octaves):
        total = total + amp * _noise3_torch(p, x * freq, y * freq, z * freq)
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return total / norm


def _raycast(scene: Scene, origin, dirs):
    """Nearest hit distance t along rays with unit camera-z component (so t
    is the camera depth) and the world hit points; torch float64."""
    import torch
    dev = dirs.device
    o = torch.as_tensor(origin, dtype=torch.float64, device=dev)   # (3,) or one per ray (n, 3)
    n = dirs.shape[0]
    t_best = torch.full((n,), float("inf"), dtype=torch.float64, device=dev)
    dy = dirs[:, 1]
    tg = (scene.cam_height - (o[1] if o.dim() == 1 else o[:, 1])) / dy
    tg = torch.where((dy > 1e-12) & (tg > 0), tg, torch.full_like(tg, float("inf")))
    t_best = torch.minimum(t_best, tg)
    inv = 1.0 / dirs
    boxes = torch.as_tensor(scene.boxes, dtype=torch.float64, device=dev)
    for b in boxes:
        t1 = (b[:3] - o) * inv
        t2 = (b[3:] - o) * inv
        lo = torch.minimum(t1, t2).nan_to_num(nan=-float("inf"))
        hi = torch.maximum(t1, t2).nan_to_num(nan=float("inf"))
        tmin = lo.max(dim=1).values
        tmax = hi.min(dim=1).values
        hit = (tmax >= tmin) & (tmax > 0)
        th = torch.where(tmin > 0, tmin, tmax)
        t_best = torch.where(hit & (th < t_best), th, t_best)
    oc = o - torch.as_tensor(scene.backdrop_center, dtype=torch.float64, device=dev)
    a = (dirs * dirs).sum(1)
    if oc.dim() == 1:
        bq = 2.0 * (dirs @ oc)
        cq = (oc @ oc) - scene.backdrop_radius ** 2
    else:
        bq = 2.0 * (dirs * oc).sum(1)
        cq = (oc * oc).sum(1) - scene.backdrop_radius ** 2
    disc = torch.clamp(bq * bq - 4.0 * a * cq, min=0.0)
    ts = (-bq + torch.sqrt(disc)) / (2.0 * a)
    t_best = torch.minimum(t_best, ts)
    return t_best, (o[None, :] if o.dim() == 1 else o) + t_best[:, None] * dirs


def render_view(scene: Scene, cam: Camera, Rwc: np.ndarray, centre: np.ndarray,
                noise_rng: np.random.Generator | None, device="cpu"):
    """Intensity image (uint8 numpy) and camera-frame depth z for one camera."""
    import torch
    yy, xx = torch.meshgrid(torch.arange(cam.h, dtype=torch.float64, device=device),
                            torch.arange(cam.w, dtype=torch.float64, device=device),
                            indexing="ij")
    d_cam = torch.stack([(xx - cam.cx) / cam.f, (yy - cam.cy) / cam.f, torch.ones_like(xx)], -1)
    dirs = d_cam.reshape(-1, 3) @ torch.as_tensor(Rwc, dtype=torch.float64, device=device).T
    t, pts = _raycast(scene, centre, dirs)
    perm = rng(scene.tex_seed).permutation(256).astype(np.int64)
    p = _perlin_torch(perm, device)
    v = 128.0 + 180.0 * _fbm3_torch(p, pts[:, 0] / 0.6, pts[:, 1] / 0.6, pts[:, 2] / 0.6)
    v = v.cpu().numpy()
    if noise_rng is not None and scene.noise_sigma > 0:
        v = v + noise_rng.normal(0.0, scene.noise_sigma, size=v.shape)
    return _to_u8(v).reshape(cam.h, cam.w), t.cpu().numpy().reshape(cam.h, cam.w)


def render_frame(scene: Scene, cam: Camera, k: int, noise: bool = True, device="cpu"):
    """Left/right uint8 images and left ground-truth disparity for frame k."""
    Rwc, c = scene.poses[k]
    nr = rng(splitmix64(scene.noise_seed + k)) if noise else None
    left, zl = render_view(scene, cam, Rwc, c, nr, device)
    cr = c + Rwc @ np.array([cam.baseline, 0.0, 0.0])
    right, _ = render_view(scene, cam, Rwc, cr, nr, device)
    gt = cam.f * cam.baseline / zl
    return left, right, gt


def render_frames_device(scene: Scene, cam: Camera, ks, device, noise: bool = True):
    """Frames ks as (left, right) uint8 device tensors, all views of the
    batch in one raycast and one texture evaluation.  The geometry and
    texture are those of render_frame; the sensor noise is drawn on the
    device (torch generator seeded per frame), so the images differ from
    render_frame's in the noise only."""
    import torch
    yy, xx = torch.meshgrid(torch.arange(cam.h, dtype=torch.float64, device=device),
                            torch.arange(cam.w, dtype=torch.float64, device=device),
                            indexing="ij")
    d_cam = torch.stack([(xx - cam.cx) / cam.f, (yy - cam.cy) / cam.f, torch.ones_like(xx)],
                        -1).reshape(-1, 3)
    n = cam.w * cam.h
    dirs, orgs = [], []
    for k in ks:
        Rwc, c = scene.poses[k]
        Rt = torch.as_tensor(Rwc, dtype=torch.float64, device=device).T
        for cc in (c, c + Rwc @ np.array([cam.baseline, 0.0, 0.0])):
            dirs.append(d_cam @ Rt)
            orgs.append(torch.as_tensor(cc, dtype=torch.float64, device=device).expand(n, 3))
    _, pts = _raycast(scene, torch.cat(orgs), torch.cat(dirs))
    perm = rng(scene.tex_seed).permutation(256).astype(np.int64)
    p = _perlin_torch(perm, device)
    v = 128.0 + 180.0 * _fbm3_torch(p, pts[:, 0] / 0.6, pts[:, 1] / 0.6, pts[:, 2] / 0.6)
    v = v.reshape(len(ks), 2, cam.h, cam.w)
    out = []
    for i, k in enumerate(ks):
        vi = v[i]
        if noise and scene.noise_sigma > 0:
            g = torch.Generator(device=device)
            g.manual_seed(int(splitmix64(scene.noise_seed + k) & 0x7FFFFFFFFFFFFFFF))
            vi = vi + scene.noise_sigma * torch.randn(vi.shape, generator=g, dtype=torch.float64,
                                                      device=device)
        u8 = torch.clamp(torch.floor(vi + 0.5), 0, 255).to(torch.uint8)
        out.append((u8[0].contiguous(), u8[1].contiguous()))
    return out


def relative_motion(scene: Scene, k: int):
    """(R, t) with M_k = R M_{k-1} + t, camera coordinates of frame k-1 to k."""
    R0, c0 = scene.poses[k - 1]
    R1, c1 = scene.poses[k]
    R = R1.T @ R0
    t = R1.T @ (c0 - c1)
    return R, t


@dataclass
class Sequence:
    cam: Camera
    scene: Scene
    n_frames: int

    def frame(self, k: int, noise: bool = True, device="cpu"):
        return render_frame(self.scene, self.cam, k, noise, device)

    def motion(self, k: int):
        return relative_motion(self.scene, k)


def street_sequence(w: int = 1242, h: int = 375, n_frames: int = 20, seed: int | None = None,
                    noise_sigma: float = 2.0, f: float | None = None) -> Sequence:
    if seed is None:
        seed = seed_for(1)
    cam = Camera.kitti_like(w, h, f)
    scene = make_scene(seed, n_frames, noise_sigma=noise_sigma)
    return Sequence(cam, scene, n_frames)
