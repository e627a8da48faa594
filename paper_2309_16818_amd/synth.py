"""Seeded synthetic terrain and sensor data.

This module only simulates the world and the sensors: a height field, a
robot walking over it, LiDAR / depth-camera point clouds and camera images.
It holds none of the map update's arithmetic (no cell association, no
fusion) and is shared by the tests, the benchmark and the smoke check.

Workloads (sizes follow the paper's scales: a ~10 m robot-centric grid at
4 cm, hundreds of thousands of points per cloud, Table I and Table II):

* ``small``  - 200x200 cells at 0.04 m, 10 frames, one 20k-point cloud per
  frame sampled on the terrain within 4 m (4 Dirichlet(1) class channels per
  point), one 320x240 camera with an RGB u8 image and an 8-class image.
* ``full``   - 500x500 cells at 0.04 m, a 128x2048 LiDAR and four 640x480
  depth cameras per frame (~1.49M points), four RGB cameras each with an RGB
  u8 image, a 160x120x64 unit-norm feature image and a 20-class image.

Terrain: a sum of 8 random sinusoids (amplitudes summing to 0.3 m,
wavelengths 1-8 m) plus 5 boxes 0.2-1.0 m wide and 0.05-0.5 m tall.  The
robot takes steps of at most 0.1 m and 5 degrees.  Point noise is added along
world z with sigma = 0.01 + 0.001 r^2 (r the range to the sensor).  All
random numbers come from numpy PCG64 seeded per workload; ray casting of the
terrain may run on a torch device but draws no random numbers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

try:  # torch is optional here: ray casting falls back to numpy
    import torch
except Exception:  # pragma: no cover
    torch = None


# --------------------------------------------------------------------------
# Terrain
# --------------------------------------------------------------------------

@dataclass
class Terrain:
    amp: np.ndarray      # (8,)
    lam: np.ndarray      # (8,)
    phi: np.ndarray      # (8,)
    psi: np.ndarray      # (8,)
    boxes: np.ndarray    # (nb, 5): centre x, centre y, half-width x, half-width y, height
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def zmax(self) -> float:
        """Upper bound of the height field."""
        return float(np.sum(np.abs(self.amp)) + (self.boxes[:, 4].max() if len(self.boxes) else 0.0))

    # -- numpy -------------------------------------------------------------
    def height(self, x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        h = np.zeros(np.broadcast(x, y).shape)
        for a, l, f, p in zip(self.amp, self.lam, self.phi, self.psi):
            h += a * np.sin(2 * np.pi * (x * np.cos(f) + y * np.sin(f)) / l + p)
        for bx, by, hx, hy, bh in self.boxes:
            inside = (np.abs(x - bx) <= hx) & (np.abs(y - by) <= hy)
            h = np.where(inside, h + bh, h)
        return h

    def albedo(self, x, y):
        """RGB in [0, 1]: grass/soil stripes, each box its own colour."""
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        g = 0.5 + 0.25 * np.sin(1.7 * x + 0.3) * np.cos(1.3 * y - 0.2)
        rgb = np.stack([0.35 + 0.3 * g, 0.45 + 0.35 * (1 - g), 0.2 + 0.1 * g], -1)
        for k, (bx, by, hx, hy, _) in enumerate(self.boxes):
            inside = (np.abs(x - bx) <= hx) & (np.abs(y - by) <= hy)
            col = np.array([0.8 * ((k + 1) % 2), 0.2 + 0.15 * k, 0.9 * (k % 3 == 0)])
            rgb = np.where(inside[..., None], col, rgb)
        return np.clip(rgb, 0, 1)

    # -- torch -------------------------------------------------------------
    def height_t(self, x, y):
        key = (x.device, x.dtype)
        if key not in self._cache:
            t = lambda a: torch.as_tensor(np.asarray(a), device=x.device, dtype=x.dtype)
            self._cache[key] = (t(self.amp), t(2 * np.pi * np.cos(self.phi) / self.lam),
                                t(2 * np.pi * np.sin(self.phi) / self.lam), t(self.psi), t(self.boxes))
        amp, kx, ky, psi, boxes = self._cache[key]
        h = torch.zeros_like(x)
        for k in range(amp.shape[0]):
            h = h + amp[k] * torch.sin(x * kx[k] + y * ky[k] + psi[k])
        for b in range(boxes.shape[0]):
            bx, by, hx, hy, bh = boxes[b]
            inside = ((x - bx).abs() <= hx) & ((y - by).abs() <= hy)
            h = h + inside.to(x.dtype) * bh
        return h


def make_terrain(rng: np.random.Generator, extent: float, n_waves: int = 8,
                 n_boxes: int = 5, amplitude: float = 0.3) -> Terrain:
    a = rng.uniform(0, 1, n_waves)
    a = amplitude * a / a.sum()
    lam = rng.uniform(1.0, 8.0, n_waves)
    phi = rng.uniform(0, 2 * np.pi, n_waves)
    psi = rng.uniform(0, 2 * np.pi, n_waves)
    boxes = []
    while len(boxes) < n_boxes:
        side = rng.uniform(0.2, 1.0, 2)
        c = rng.uniform(-extent / 2, extent / 2, 2)
        if np.hypot(*c) < 0.5 + side.max():  # keep the start clear
            continue
        boxes.append([c[0], c[1], side[0] / 2, side[1] / 2, rng.uniform(0.05, 0.5)])
    return Terrain(a, lam, phi, psi, np.array(boxes).reshape(-1, 5))


# --------------------------------------------------------------------------
# Poses
# --------------------------------------------------------------------------

def rot_z(yaw: float) -> np.ndarray:
    c, s = math.cos(yaw), math.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def camera_rotation(yaw: float, pitch_down: float) -> np.ndarray:
    """Camera -> map rotation; camera x right, y down, z forward."""
    cp, sp = math.cos(pitch_down), math.sin(pitch_down)
    cy, sy = math.cos(yaw), math.sin(yaw)
    z = np.array([cy * cp, sy * cp, -sp])
    x = np.array([sy, -cy, 0.0])
    y = np.cross(z, x)
    return np.stack([x, y, z], 1)


def pose_matrix(R: np.ndarray, t) -> np.ndarray:
    T = np.zeros((3, 4), np.float32)
    T[:, :3] = R
    T[:, 3] = t
    return T


def pose_walk(rng: np.random.Generator, n: int, step: float = 0.1,
              dyaw_deg: float = 5.0):
    """Random walk from (0, 0, yaw 0): each step moves up to `step` metres
    (uniform in a disc) and turns up to `dyaw_deg` degrees."""
    x = y = yaw = 0.0
    out = []
    for i in range(n):
        if i > 0:
            r = step * math.sqrt(rng.uniform())
            a = rng.uniform(0, 2 * np.pi)
            x += r * math.cos(a)
            y += r * math.sin(a)
            yaw += math.radians(rng.uniform(-dyaw_deg, dyaw_deg))
        out.append((x, y, yaw))
    return out


# --------------------------------------------------------------------------
# Ray casting the terrain
# --------------------------------------------------------------------------

def raycast(ter: Terrain, o, d, tmax: float, step: float = 0.04, tmin: float = 0.05,
            refine: int = 12, device=None):
    """First hit of rays o + t d (|d| = 1) with the height field, t <= tmax.
    Returns t (NaN for a miss).  Runs on torch `device` if given."""
    zmax = ter.zmax
    if device is not None and torch is not None:
        dt = torch.float32 if str(device).startswith("cuda") else torch.float64
        O = torch.as_tensor(np.array(o), device=device, dtype=dt)
        D = torch.as_tensor(np.array(d), device=device, dtype=dt)
        f = lambda t: O[:, 2] + t * D[:, 2] - ter.height_t(O[:, 0] + t * D[:, 0], O[:, 1] + t * D[:, 1])
        lo = torch.full(O.shape[:1], tmin, device=device, dtype=dt)
        hit = torch.full_like(lo, float("nan"))
        hi_t = torch.full_like(lo, float("nan"))
        # the sample positions t -> t2 of the march, in the order taken
        steps = []
        t = tmin
        while t < tmax:
            t2 = min(t + step, tmax)
            steps.append((t, t2))
            t = t2
        prev_above = f(lo) > 0
        # blocks of `chunk` samples per launch: a ray stops at its first
        # sample below the terrain (a crossing in [t, t2]) or where it has
        # left the height field's bounding slab upwards
        chunk = 32
        for b0 in range(0, len(steps), chunk):
            blk = steps[b0:b0 + chunk]
            T0 = torch.tensor([a for a, _ in blk], device=device, dtype=dt)
            T2 = torch.tensor([b for _, b in blk], device=device, dtype=dt)
            idx = torch.nonzero(prev_above).squeeze(1)
            if idx.numel() == 0:
                break
            Oi, Di = O[idx], D[idx]
            x = Oi[:, 0:1] + T2[None, :] * Di[:, 0:1]
            y = Oi[:, 1:2] + T2[None, :] * Di[:, 1:2]
            val = Oi[:, 2:3] + T2[None, :] * Di[:, 2:3] - ter.height_t(x, y)
            cross = val <= 0
            escaped = (Di[:, 2:3] >= 0) & (Oi[:, 2:3] + T2[None, :] * Di[:, 2:3] > zmax)
            stop = cross | escaped
            any_stop = stop.any(1)
            first = torch.argmax(stop.to(torch.int8), 1)
            crossed = any_stop & cross.gather(1, first[:, None]).squeeze(1)
            ci = idx[crossed]
            lo[ci] = T0[first[crossed]]
            hi_t[ci] = T2[first[crossed]]
            prev_above[idx[any_stop]] = False
        m = ~torch.isnan(hi_t)
        a, b = lo[m], hi_t[m]
        Om, Dm = O[m], D[m]
        fm = lambda tt: Om[:, 2] + tt * Dm[:, 2] - ter.height_t(Om[:, 0] + tt * Dm[:, 0], Om[:, 1] + tt * Dm[:, 1])
        for _ in range(refine):
            c = 0.5 * (a + b)
            above = fm(c) > 0
            a = torch.where(above, c, a)
            b = torch.where(above, b, c)
        hit[m] = 0.5 * (a + b)
        return hit.cpu().numpy().astype(np.float64)
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    f = lambda t, idx=slice(None): o[idx, 2] + t * d[idx, 2] - ter.height(o[idx, 0] + t * d[idx, 0], o[idx, 1] + t * d[idx, 1])
    n = o.shape[0]
    lo = np.full(n, tmin)
    hi = np.full(n, np.nan)
    active = f(lo) > 0
    t = tmin
    while t < tmax and active.any():
        t2 = min(t + step, tmax)
        idx = np.nonzero(active)[0]
        val = f(t2, idx)
        cr = val <= 0
        lo[idx[cr]] = t
        hi[idx[cr]] = t2
        active[idx[cr]] = False
        gone = (d[idx, 2] >= 0) & (o[idx, 2] + t2 * d[idx, 2] > zmax)
        active[idx[gone]] = False
        t = t2
    m = ~np.isnan(hi)
    idx = np.nonzero(m)[0]
    a, b = lo[idx], hi[idx]
    for _ in range(refine):
        c = 0.5 * (a + b)
        above = f(c, idx) > 0
        a = np.where(above, c, a)
        b = np.where(above, b, c)
    out = np.full(n, np.nan)
    out[idx] = 0.5 * (a + b)
    return out


def segment_clear(ter: Terrain, o, p, samples: int = 32, eps: float = 1e-3) -> np.ndarray:
    """True where the straight segment from o to each p stays above the
    terrain (the point is visible from o)."""
    o = np.asarray(o, np.float64).reshape(1, 3)
    p = np.asarray(p, np.float64)
    t = (np.arange(1, samples) / samples).reshape(1, -1)
    x = o[:, 0:1] + t * (p[:, 0:1] - o[:, 0:1])
    y = o[:, 1:2] + t * (p[:, 1:2] - o[:, 1:2])
    z = o[:, 2:3] + t * (p[:, 2:3] - o[:, 2:3])
    return np.all(ter.height(x, y) < z - eps, axis=1)


def add_noise(rng: np.random.Generator, p: np.ndarray, origin, c0=0.01, c1=0.001) -> np.ndarray:
    r2 = np.sum((p - np.asarray(origin).reshape(1, 3)) ** 2, 1)
    q = p.copy()
    q[:, 2] += rng.standard_normal(p.shape[0]) * (c0 + c1 * r2)
    return q


def to_sensor(p_map: np.ndarray, T: np.ndarray) -> np.ndarray:
    R = T[:, :3].astype(np.float64)
    t = T[:, 3].astype(np.float64)
    return ((p_map - t) @ R).astype(np.float32)


# --------------------------------------------------------------------------
# Sensors
# --------------------------------------------------------------------------

def disc_cloud(rng, ter: Terrain, sensor_xyz, yaw: float, n: int, radius: float = 4.0):
    """n visible terrain points uniform in a disc around the sensor, with
    noise; returns (points in the sensor frame, T_map_sensor)."""
    T = pose_matrix(rot_z(yaw), sensor_xyz)
    pts = []
    got = 0
    while got < n:
        m = int((n - got) * 1.4) + 64
        r = radius * np.sqrt(rng.uniform(size=m))
        a = rng.uniform(0, 2 * np.pi, m)
        x = sensor_xyz[0] + r * np.cos(a)
        y = sensor_xyz[1] + r * np.sin(a)
        p = np.stack([x, y, ter.height(x, y)], 1)
        p = p[segment_clear(ter, sensor_xyz, p)]
        pts.append(p)
        got += p.shape[0]
    p = np.concatenate(pts)[:n]
    p = add_noise(rng, p, sensor_xyz)
    return to_sensor(p, T), T


def depth_camera_cloud(rng, ter, T_cam: np.ndarray, K, h: int, w: int, tmax: float, device=None):
    """Back-projected depth image (row-major pixel order), misses dropped."""
    fx, fy, cx, cy = K
    v, u = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    d = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u, dtype=np.float64)], -1).reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    R = T_cam[:, :3].astype(np.float64)
    o = T_cam[:, 3].astype(np.float64)
    dm = d @ R.T
    t = raycast(ter, np.broadcast_to(o, dm.shape), dm, tmax, device=device)
    ok = ~np.isnan(t)
    p = o + t[ok, None] * dm[ok]
    p = add_noise(rng, p, o)
    return to_sensor(p, T_cam)


def lidar_cloud(rng, ter, T_lidar: np.ndarray, beams: int, azimuths: int,
                el_min_deg: float, el_max_deg: float, tmax: float, device=None):
    """Spinning LiDAR, azimuth-major order (all beams of one firing, then the
    next azimuth); misses dropped."""
    el = np.radians(np.linspace(el_min_deg, el_max_deg, beams))
    az = np.arange(azimuths) * (2 * np.pi / azimuths)
    A, E = np.meshgrid(az, el, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1).reshape(-1, 3)
    R = T_lidar[:, :3].astype(np.float64)
    o = T_lidar[:, 3].astype(np.float64)
    dm = d @ R.T
    t = raycast(ter, np.broadcast_to(o, dm.shape), dm, tmax, device=device)
    ok = ~np.isnan(t)
    p = o + t[ok, None] * dm[ok]
    p = add_noise(rng, p, o)
    return to_sensor(p, T_lidar)


def render_rgb(ter: Terrain, T_cam, K, h: int, w: int, tmax: float, device=None,
               step: float = 0.06) -> np.ndarray:
    fx, fy, cx, cy = K
    v, u = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    d = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u, dtype=np.float64)], -1).reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    R = T_cam[:, :3].astype(np.float64)
    o = T_cam[:, 3].astype(np.float64)
    dm = d @ R.T
    t = raycast(ter, np.broadcast_to(o, dm.shape), dm, tmax, step=step, refine=8, device=device)
    rgb = np.tile(np.array([0.53, 0.81, 0.92]), (h * w, 1))  # sky
    ok = ~np.isnan(t)
    p = o + t[ok, None] * dm[ok]
    rgb[ok] = ter.albedo(p[:, 0], p[:, 1])
    return np.round(rgb * 255).astype(np.uint8).reshape(h, w, 3)


def class_image(rng, h: int, w: int, k: int) -> np.ndarray:
    """Per-pixel Dirichlet(1) class probabilities (normalised Exp(1))."""
    e = rng.standard_exponential((h, w, k), dtype=np.float32)
    return (e / e.sum(-1, keepdims=True)).astype(np.float32)


def feature_image(rng, h: int, w: int, c: int) -> np.ndarray:
    """Per-pixel N(0, I) features normalised to unit length."""
    f = rng.standard_normal((h, w, c), dtype=np.float32)
    return (f / np.linalg.norm(f, axis=-1, keepdims=True)).astype(np.float32)


def scaled_intrinsics(K, s: float):
    """Intrinsics of the same camera at s times the resolution (pixel
    centres at integers)."""
    fx, fy, cx, cy = K
    return (fx * s, fy * s, (cx + 0.5) * s - 0.5, (cy + 0.5) * s - 0.5)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

SMALL_MAP = dict(width=200, height=200, resolution=0.04, noise_c0=0.01, noise_c1=0.001,
                 max_range=10.0, clear_margin=0.05, clear_min_count=1, min_depth=0.1)
# layers: point classes (Dirichlet K=4), RGB (exp. averaging w=0.5), image classes (Dirichlet K=8)
SMALL_LAYERS = [(4, 3, 1.0), (3, 1, 0.5), (8, 3, 1.0)]

FULL_MAP = dict(width=500, height=500, resolution=0.04, noise_c0=0.01, noise_c1=0.001,
                max_range=15.0, clear_margin=0.05, clear_min_count=1, min_depth=0.1)
# layers: RGB (exp. averaging), 64-d features (Gaussian, sigma_f^2 = 1), 20 classes (Dirichlet)
FULL_LAYERS = [(3, 1, 0.5), (64, 2, 1.0), (20, 3, 1.0)]


def small_frames(seed: int = 0, n_frames: int = 10, n_points: int = 20000,
                 cam_hw=(240, 320), device=None):
    """The small workload: list of frames, each a dict with
    pose (x, y, yaw), cloud (xyz, ch, T), camera (K, T, rgb, classes)."""
    ss = np.random.SeedSequence(seed)
    rng_t, rng_p, rng_f = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    ter = make_terrain(rng_t, extent=8.0)
    poses = pose_walk(rng_p, n_frames)
    frames = []
    h, w = cam_hw
    K = (200.0, 200.0, (w - 1) / 2.0, (h - 1) / 2.0)
    for (x, y, yaw) in poses:
        zg = float(ter.height(x, y))
        s = np.array([x, y, zg + 0.6])
        xyz, T = disc_cloud(rng_f, ter, s, yaw, n_points)
        ch = class_image(rng_f, 1, n_points, 4).reshape(n_points, 4)
        Tc = pose_matrix(camera_rotation(yaw, math.radians(20)), s)
        rgb = render_rgb(ter, Tc, K, h, w, tmax=8.0, device=device)
        cls = class_image(rng_f, h, w, 8)
        frames.append(dict(pose=(x, y, yaw), cloud=dict(xyz=xyz, ch=ch, T=T),
                           camera=dict(K=K, T=Tc, rgb=rgb, classes=cls)))
    return ter, frames


def full_frames(seed: int = 1, n_frames: int = 2, device=None, **kw):
    """The full-rate single-robot workload (see module docstring)."""
    frames = list(iter_full_frames(seed, n_frames, device, **kw))
    return frames[0][0] if frames else None, [f for _, f in frames]


def iter_full_frames(seed: int = 1, n_frames: int = 2, device=None, lidar=(128, 2048),
                     depth_hw=(480, 640), rgb_hw=(480, 640), feat_hw=(120, 160), n_feat=64,
                     n_cls=20):
    """Yields (terrain, frame) of the full-rate single-robot workload one
    frame at a time."""
    ss = np.random.SeedSequence(seed)
    rng_t, rng_p, rng_f = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    ter = make_terrain(rng_t, extent=20.0)
    poses = pose_walk(rng_p, n_frames)
    dh, dw = depth_hw
    Kd = (400.0, 400.0, (dw - 1) / 2.0, (dh - 1) / 2.0)
    rh, rw = rgb_hw
    Kr = (400.0, 400.0, (rw - 1) / 2.0, (rh - 1) / 2.0)
    Kf = scaled_intrinsics(Kr, feat_hw[1] / rw)
    for (x, y, yaw) in poses:
        zg = float(ter.height(x, y))
        base = np.array([x, y, zg])
        clouds = []
        Tl = pose_matrix(rot_z(yaw), base + [0, 0, 0.8])
        clouds.append(dict(xyz=lidar_cloud(rng_f, ter, Tl, lidar[0], lidar[1], -25.0, -1.0, 14.1,
                                           device=device), T=Tl))
        cams = []
        for k in range(4):
            Tc = pose_matrix(camera_rotation(yaw + k * np.pi / 2, math.radians(25)), base + [0, 0, 0.6])
            clouds.append(dict(xyz=depth_camera_cloud(rng_f, ter, Tc, Kd, dh, dw, 10.0, device=device), T=Tc))
            cams.append(dict(T=Tc, K=Kr, rgb=render_rgb(ter, Tc, Kr, rh, rw, 10.0, device=device),
                             classes=class_image(rng_f, rh, rw, n_cls),
                             K_feat=Kf, features=feature_image(rng_f, feat_hw[0], feat_hw[1], n_feat)))
        yield ter, dict(pose=(x, y, yaw), clouds=clouds, cameras=cams)


# --------------------------------------------------------------------------
# Batched workload: many robots, each with its own terrain and map
# --------------------------------------------------------------------------

BATCH_RES = 0.05
BATCH_CAM = dict(h=96, w=128, fx=80.0, fy=80.0, cx=63.5, cy=47.5, c=16)


class BatchWorld:
    """n robots on n seeded terrains (8 sinusoids with amplitudes summing to
    0.3 m, wavelengths 1-8 m, plus 5 boxes each), map sides uniform in
    [side_lo, side_hi] cells at 0.05 m, point counts per step uniform in
    [pts_lo, pts_hi], sampled in a disc of radius min(4 m, half the map)
    around the sensor (0.6 m up) on the terrain, with z-noise
    0.01 + 0.001 r^2; one 128x96 camera per robot (fx 80, pitched 30 deg
    down, 0.7 m up) with 16 unit-norm Gaussian feature channels.  Points are
    not tested for occlusion (every sample is taken as seen).  Generation
    runs on a torch device."""

    def __init__(self, n=1024, seed=3, side_lo=64, side_hi=256, pts_lo=4000, pts_hi=60000, device="cuda"):
        self.n, self.device = n, device
        ss = np.random.SeedSequence(seed)
        self.rng = np.random.Generator(np.random.PCG64(ss.spawn(1)[0]))
        r = self.rng
        self.side = r.integers(side_lo, side_hi + 1, n)
        self.pts_lo, self.pts_hi = pts_lo, pts_hi
        a = r.uniform(0, 1, (n, 8))
        a = 0.3 * a / a.sum(1, keepdims=True)
        lam = r.uniform(1, 8, (n, 8))
        phi = r.uniform(0, 2 * np.pi, (n, 8))
        t = lambda v: torch.as_tensor(v, dtype=torch.float32, device=device)
        self.amp, self.psi = t(a), t(r.uniform(0, 2 * np.pi, (n, 8)))
        self.kx, self.ky = t(2 * np.pi * np.cos(phi) / lam), t(2 * np.pi * np.sin(phi) / lam)
        ext = self.side * BATCH_RES
        bc = r.uniform(-0.5, 0.5, (n, 5, 2)) * ext[:, None, None]
        bh = r.uniform(0.1, 0.5, (n, 5, 2))
        self.box = t(np.concatenate([bc, bh, r.uniform(0.05, 0.5, (n, 5, 1))], -1))  # cx cy hx hy h
        self.pose = np.zeros((n, 3))
        self.pose[:, 2] = r.uniform(0, 2 * np.pi, n)

    def height(self, mid, x, y):
        h = torch.zeros_like(x)
        for k in range(8):
            h = h + self.amp[mid, k] * torch.sin(x * self.kx[mid, k] + y * self.ky[mid, k] + self.psi[mid, k])
        for b in range(5):
            B = self.box[mid, b]
            inside = ((x - B[:, 0]).abs() <= B[:, 2]) & ((y - B[:, 1]).abs() <= B[:, 3])
            h = h + inside.float() * B[:, 4]
        return h

    def step(self, k):
        """Advances every robot and returns one step's inputs (device xyz,
        host offsets / poses / cameras)."""
        r = self.rng
        n = self.n
        if k > 0:
            d = 0.1 * np.sqrt(r.uniform(size=n))
            a = r.uniform(0, 2 * np.pi, n)
            self.pose[:, 0] += d * np.cos(a)
            self.pose[:, 1] += d * np.sin(a)
            self.pose[:, 2] += np.radians(r.uniform(-5, 5, n))
        cnt = r.integers(self.pts_lo, self.pts_hi + 1, n)
        offs = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        dev = self.device
        mid = torch.repeat_interleave(torch.arange(n, device=dev), torch.as_tensor(cnt, device=dev))
        radius = torch.as_tensor(np.minimum(4.0, 0.5 * self.side * BATCH_RES), dtype=torch.float32, device=dev)
        g = torch.Generator(device=dev)
        g.manual_seed(int(r.integers(0, 2**62)))
        u = torch.rand(int(offs[-1]), 4, device=dev, generator=g)
        px0 = torch.as_tensor(self.pose[:, 0], dtype=torch.float32, device=dev)[mid]
        py0 = torch.as_tensor(self.pose[:, 1], dtype=torch.float32, device=dev)[mid]
        rr = radius[mid] * u[:, 0].sqrt()
        ang = u[:, 1] * (2 * np.pi)
        x = px0 + rr * torch.cos(ang)
        y = py0 + rr * torch.sin(ang)
        ground0 = self.height(torch.arange(n, device=dev), torch.as_tensor(self.pose[:, 0], dtype=torch.float32, device=dev),
                              torch.as_tensor(self.pose[:, 1], dtype=torch.float32, device=dev))
        sz = ground0 + 0.6
        z = self.height(mid, x, y)
        rng3 = torch.sqrt((x - px0) ** 2 + (y - py0) ** 2 + (z - sz[mid]) ** 2)
        z = z + torch.randn(z.shape, device=dev, generator=g) * (0.01 + 0.001 * rng3 ** 2)
        yaw = torch.as_tensor(self.pose[:, 2], dtype=torch.float32, device=dev)[mid]
        dx, dy, dz = x - px0, y - py0, z - sz[mid]
        c, s = torch.cos(yaw), torch.sin(yaw)
        xyz = torch.stack([c * dx + s * dy, -s * dx + c * dy, dz], 1).contiguous()
        g0 = ground0.cpu().numpy()
        T = np.zeros((n, 3, 4), np.float32)
        Tc = np.zeros((n, 3, 4), np.float32)
        for m in range(n):
            T[m] = pose_matrix(rot_z(self.pose[m, 2]), (self.pose[m, 0], self.pose[m, 1], g0[m] + 0.6))
            Tc[m] = pose_matrix(camera_rotation(self.pose[m, 2], math.radians(30)),
                                (self.pose[m, 0], self.pose[m, 1], g0[m] + 0.7))
        cam = BATCH_CAM
        K = np.tile(np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"]], np.float32), (n, 1))
        return dict(xyz=xyz, offsets=offs, T=T, T_cam=Tc, K=K,
                    robot_xy=self.pose[:, :2].astype(np.float32).copy())

    def images(self, seed):
        cam = BATCH_CAM
        g = torch.Generator(device=self.device)
        g.manual_seed(seed)
        f = torch.randn(self.n, cam["h"], cam["w"], cam["c"], device=self.device, generator=g)
        return (f / f.norm(dim=-1, keepdim=True)).contiguous()


# --------------------------------------------------------------------------
# Completion pairs: dense 360-degree sweeps against one forward sensor
# --------------------------------------------------------------------------

class CompletionWorld:
    """n windows of `size` cells at `res` metres, each on its own seeded
    terrain (8 sinusoids with amplitudes summing to 0.3 m, wavelengths 1-8 m,
    and 5 boxes 0.2-1.0 m wide, 0.05-0.5 m tall inside the window), with the
    robot at the window centre (the origin) under a random yaw, its sensors
    0.6 m above the ground there.

    * ``dense_step(v)`` (v = 0..4): a 360-degree sweep from viewpoint v (the
      centre, then four points at +-0.3 of the window side in x and y):
      1.5 points per cell drawn uniformly over the window, kept if within
      0.6 window sides of the viewpoint and visible from it (the straight
      segment stays above the terrain at 15 samples).
    * ``sparse_step()``: one forward sensor at the centre, a 90-degree
      sector around the yaw, ranges 0.3 m to 0.45 window sides, the same
      density, visible points only, minus the shadows of 2-5 random vertical
      cylinders (radius 0.1-0.4 m, 1-4 m ahead inside the sector), which
      stand in for transient obstacles and are not part of the terrain.

    Points get z-noise 0.01 + 0.001 r^2 for range r to their sensor and are
    returned in that sensor's frame.  All random numbers come from numpy
    PCG64 (terrain, poses, occluders) and a seeded torch generator on the
    device (point samples, noise)."""

    VIEW = ((0.0, 0.0), (0.3, 0.0), (-0.3, 0.0), (0.0, 0.3), (0.0, -0.3))

    def __init__(self, n, size=256, res=0.04, seed=0, device="cuda"):
        self.n, self.size, self.res, self.device = n, size, res, device
        self.ext = size * res
        r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, n, size])))
        self.rng = r
        a = r.uniform(0, 1, (n, 8))
        a = 0.3 * a / a.sum(1, keepdims=True)
        lam = r.uniform(1, 8, (n, 8))
        phi = r.uniform(0, 2 * np.pi, (n, 8))
        t = lambda v: torch.as_tensor(v, dtype=torch.float32, device=device)
        self.amp, self.psi = t(a), t(r.uniform(0, 2 * np.pi, (n, 8)))
        self.kx, self.ky = t(2 * np.pi * np.cos(phi) / lam), t(2 * np.pi * np.sin(phi) / lam)
        bc = r.uniform(-0.45, 0.45, (n, 5, 2)) * self.ext
        bh = r.uniform(0.1, 0.5, (n, 5, 2))
        self.box = t(np.concatenate([bc, bh, r.uniform(0.05, 0.5, (n, 5, 1))], -1))
        self.yaw = r.uniform(0, 2 * np.pi, n)
        ids = torch.arange(n, device=device)
        zero = torch.zeros(n, device=device)
        self.ground = self.height(ids, zero, zero).cpu().numpy().astype(np.float64)
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(int(r.integers(0, 2**62)))

    def height(self, mid, x, y):
        h = torch.zeros_like(x)
        for k in range(8):
            h = h + self.amp[mid, k] * torch.sin(x * self.kx[mid, k] + y * self.ky[mid, k] + self.psi[mid, k])
        for b in range(5):
            B = self.box[mid, b]
            inside = ((x - B[:, 0]).abs() <= B[:, 2]) & ((y - B[:, 1]).abs() <= B[:, 3])
            h = h + inside.float() * B[:, 4]
        return h

    def _visible(self, mid, ox, oy, oz, x, y, z, samples=15, chunk=1 << 21):
        keep = torch.empty(x.shape, dtype=torch.bool, device=self.device)
        for s0 in range(0, x.shape[0], chunk):
            sl = slice(s0, s0 + chunk)
            ok = torch.ones(x[sl].shape, dtype=torch.bool, device=self.device)
            for k in range(1, samples + 1):
                f = k / (samples + 1)
                xs = ox[sl] + f * (x[sl] - ox[sl])
                ys = oy[sl] + f * (y[sl] - oy[sl])
                zs = oz[sl] + f * (z[sl] - oz[sl])
                ok &= self.height(mid[sl], xs, ys) < zs - 1e-3
            keep[sl] = ok
        return keep

    def _cloud(self, mid, x, y, ox, oy, oz, yaw):
        """Noisy visible points (sensor frame) and per-map offsets."""
        z = self.height(mid, x, y)
        vis = self._visible(mid, ox[mid], oy[mid], oz[mid], x, y, z)
        mid, x, y, z = mid[vis], x[vis], y[vis], z[vis]
        dx, dy, dz = x - ox[mid], y - oy[mid], z - oz[mid]
        r2 = dx * dx + dy * dy + dz * dz
        dz = dz + torch.randn(dz.shape, device=self.device, generator=self.gen) * (0.01 + 0.001 * r2)
        c, s = torch.cos(yaw)[mid], torch.sin(yaw)[mid]
        xyz = torch.stack([c * dx + s * dy, -s * dx + c * dy, dz], 1).contiguous()
        cnt = torch.bincount(mid, minlength=self.n).cpu().numpy()
        offs = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        return xyz, offs

    def _poses(self, ox, oy, oz):
        T = np.zeros((self.n, 3, 4), np.float32)
        for m in range(self.n):
            T[m] = pose_matrix(rot_z(self.yaw[m]), (ox[m], oy[m], oz[m]))
        return T

    def _common(self, per_cell):
        n, dev = self.n, self.device
        cnt = int(per_cell * self.size * self.size)
        mid = torch.arange(n, device=dev).repeat_interleave(cnt)
        u = torch.rand(n * cnt, 2, device=dev, generator=self.gen)
        return mid, (u[:, 0] - 0.5) * self.ext, (u[:, 1] - 0.5) * self.ext

    def dense_step(self, v):
        """One viewpoint's sweep for every window: dict(xyz, offsets, T, robot_xy)."""
        dev = self.device
        fx, fy = self.VIEW[v]
        vx = np.full(self.n, fx * self.ext)
        vy = np.full(self.n, fy * self.ext)
        ids = torch.arange(self.n, device=dev)
        tv = lambda a: torch.as_tensor(a, dtype=torch.float32, device=dev)
        vz = self.height(ids, tv(vx), tv(vy)).cpu().numpy() + 0.6
        mid, x, y = self._common(1.5)
        ox, oy, oz = tv(vx), tv(vy), tv(vz)
        near = (x - ox[mid]) ** 2 + (y - oy[mid]) ** 2 <= (0.6 * self.ext) ** 2
        xyz, offs = self._cloud(mid[near], x[near], y[near], ox, oy, oz, tv(self.yaw))
        return dict(xyz=xyz, offsets=offs, T=self._poses(vx, vy, vz),
                    robot_xy=np.zeros((self.n, 2), np.float32))

    def sparse_step(self):
        """The forward sensor's cloud for every window (same keys)."""
        dev, n, r = self.device, self.n, self.rng
        tv = lambda a: torch.as_tensor(a, dtype=torch.float32, device=dev)
        oz = self.ground + 0.6
        rmax = 0.45 * self.ext
        mid, x, y = self._common(1.5)
        yaw = tv(self.yaw)
        ang = torch.atan2(y, x) - yaw[mid]
        ang = torch.remainder(ang + np.pi, 2 * np.pi) - np.pi
        rr = torch.sqrt(x * x + y * y)
        keep = (ang.abs() <= np.pi / 4) & (rr >= 0.3) & (rr <= rmax)
        # occluders: k cylinders per window
        k = r.integers(2, 6, n)
        oc = np.zeros((n, 5, 3))  # x, y, radius (radius 0 = none)
        for m in range(n):
            for j in range(k[m]):
                d, a = r.uniform(1.0, 4.0), self.yaw[m] + r.uniform(-np.pi / 4, np.pi / 4)
                oc[m, j] = (d * np.cos(a), d * np.sin(a), r.uniform(0.1, 0.4))
        oc = tv(oc)
        for j in range(5):
            cx, cy, cr = oc[mid, j, 0], oc[mid, j, 1], oc[mid, j, 2]
            # closest approach of the segment origin -> point to the cylinder axis
            tt = torch.clamp((cx * x + cy * y) / torch.clamp(rr * rr, min=1e-9), 0, 1)
            dist2 = (tt * x - cx) ** 2 + (tt * y - cy) ** 2
            keep &= ~((cr > 0) & (dist2 <= cr * cr))
        zero = np.zeros(n)
        xyz, offs = self._cloud(mid[keep], x[keep], y[keep], tv(zero), tv(zero), tv(oz), yaw)
        return dict(xyz=xyz, offsets=offs, T=self._poses(zero, zero, oz),
                    robot_xy=np.zeros((n, 2), np.float32))
