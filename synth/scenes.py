"""Seeded synthetic organized point clouds (range images).

These frames stand in for the RealSense RGBD, SynPEB LiDAR and KITTI-style
recordings the paper evaluates on (Sec. 9.2-9.3, Tables 8, 11-13); none of those
datasets is used.  Each generator is deterministic in its seed and returns a
float32 array ``[M, N, 3]`` in row-major order; a missing measurement is NaN in
all three coordinates, which is how the paper marks invalid pixels (Sec. 4.2).

This module only draws inputs.  It holds none of the meshing or smoothing
arithmetic and is imported by both the oracle tests and the GPU path's tests and
benchmark.

Scene recipes
-------------
``rgbd_small`` (120x160)
    Pinhole camera, fx = fy = 140, principal point at the image centre, camera
    frame x right / y down / z forward.  A floor plane at perpendicular distance
    1.5 m whose normal is tilted 10 deg from the optical axis about x, and a
    0.3 m cube resting on the floor where the optical axis meets it, aligned with
    the floor.  Depth noise z += N(0, 2 mm) followed by back-projection along the
    pixel ray.  Exactly round(0.05 P) pixels set to NaN, uniformly at random.
``rgbd`` (480x640)
    fx = fy = 525, principal point (319.5, 239.5).  Camera 1.2 m above the floor,
    pitched 20 deg down and yawed toward a room corner formed by two orthogonal
    walls 2.2-3.8 m away, so every ray hits a surface.  Six boxes with sides
    U(0.1, 0.5) m and random yaw stand on the floor.  Depth noise
    sigma = 0.0012 z^2 m.  Random 4-connected blobs of U{5..20} pixels are cut
    out until exactly round(0.08 P) pixels are NaN.
``lidar`` (64x1024) and ``lidar128`` (128x2048)
    Spinning-LiDAR range image: elevations uniformly spaced from +3 deg (row 0)
    to -25 deg (last row), azimuth 360 deg * j / N.  Sensor 1.73 m above a road
    plane (x forward, y left, z up); sidewalks 0.15 m higher for |y| > 4 m with
    vertical curb faces; ten 4.5 x 1.8 x 1.5 m boxes at uniform random positions
    within 40 m (outside a keep-out around the sensor), random yaw.  First-hit
    ray casting, range noise N(0, 2 cm), no hit within 120 m -> NaN, then
    round(0.10 P) of the valid pixels dropped out at random.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "FrameKind", "KINDS", "make_frame", "config_frame", "random_grid",
    "batch_mix", "poisson_arrivals", "scene_planes",
]


@dataclass(frozen=True)
class FrameKind:
    name: str
    M: int
    N: int
    kernel_lap: int
    iters_lap: int
    kernel_bil: int
    iters_bil: int
    lam: float = 1.0
    sigma_length: float = 0.1
    sigma_angle: float = 0.1
    l_max: float = 0.05
    ang_min: float = 0.96


# Filter parameters per workload.  lambda = 1 and sigma_length = sigma_angle =
# 0.1 follow the parameter tables the paper uses for its OPC runs (Tables 7, 9).
# Group assignment takes l_max and ang_min from the paper's RealSense table
# (Table 7: 0.05 m, 0.96) for the pinhole frames and from its KITTI table
# (Table 4: 1.25 m, 0.97) for the LiDAR frames.
KINDS = {
    "rgbd_small": FrameKind("rgbd_small", 120, 160, 3, 3, 3, 2),
    "rgbd": FrameKind("rgbd", 480, 640, 3, 4, 3, 2),
    "lidar": FrameKind("lidar", 64, 1024, 5, 4, 5, 3, l_max=1.25, ang_min=0.97),
    "lidar128": FrameKind("lidar128", 128, 2048, 5, 4, 5, 3, l_max=1.25, ang_min=0.97),
}

# Workload index -> frame kind (the seed of frame f of workload c is 1000 c + f).
CONFIG_KIND = {0: "rgbd_small", 1: "rgbd", 2: "lidar"}


def _safe_div(a, b):
    b = np.where(b == 0.0, 1e-30, b)
    return a / b


def _ray_box(orig, dirs, center, yaw, half):
    """First positive hit distance of rays with an upright box rotated by yaw
    about the third axis (inf where missed).  orig [3], dirs [R,3]."""
    c, s = math.cos(yaw), math.sin(yaw)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])  # box->world
    o = rot.T @ (np.asarray(orig, dtype=np.float64) - center)
    d = dirs @ rot  # world->box for row vectors
    half = np.asarray(half, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        t1 = _safe_div(-half - o, d)
        t2 = _safe_div(half - o, d)
    tmin = np.max(np.minimum(t1, t2), axis=1)
    tmax = np.min(np.maximum(t1, t2), axis=1)
    hit = (tmax >= np.maximum(tmin, 0.0)) & (tmin > 1e-6)
    return np.where(hit, tmin, np.inf)


def _ray_box_frame(orig, dirs, origin, axes, lo, hi):
    """Hit distance against a box given in an arbitrary orthonormal frame:
    points q with lo <= axes @ (q - origin) <= hi componentwise."""
    o = axes @ (np.asarray(orig, dtype=np.float64) - origin)
    d = dirs @ axes.T
    with np.errstate(invalid="ignore", divide="ignore"):
        t1 = _safe_div(lo - o, d)
        t2 = _safe_div(hi - o, d)
    tmin = np.max(np.minimum(t1, t2), axis=1)
    tmax = np.min(np.maximum(t1, t2), axis=1)
    hit = (tmax >= np.maximum(tmin, 0.0)) & (tmin > 1e-6)
    return np.where(hit, tmin, np.inf)


def _pinhole_dirs(M, N, fx, fy, cx, cy):
    rows, cols = np.meshgrid(np.arange(M, dtype=np.float64),
                             np.arange(N, dtype=np.float64), indexing="ij")
    d = np.stack([(cols - cx) / fx, (rows - cy) / fy, np.ones_like(rows)], axis=-1)
    return d.reshape(-1, 3)


def _nan_uniform(pts, count, rng):
    flat = pts.reshape(-1, 3)
    idx = rng.choice(flat.shape[0], size=count, replace=False)
    flat[idx] = np.nan


_SMALL_TILT = math.radians(10.0)


def _rgbd_small(seed: int) -> np.ndarray:
    k = KINDS["rgbd_small"]
    M, N = k.M, k.N
    rng = np.random.default_rng(seed)
    fx = fy = 140.0
    cx, cy = (N - 1) / 2.0, (M - 1) / 2.0
    d = _pinhole_dirs(M, N, fx, fy, cx, cy)
    tilt = _SMALL_TILT
    n_f = np.array([0.0, -math.sin(tilt), -math.cos(tilt)])  # floor normal toward camera
    dist = 1.5
    # floor: n_f . p = -dist
    denom = d @ n_f
    t_floor = np.where(denom < 0, -dist / np.where(denom < 0, denom, -1.0), np.inf)
    # cube resting on the floor where the optical axis meets it
    hit0 = np.array([0.0, 0.0, dist / math.cos(tilt)])
    e1 = np.array([1.0, 0.0, 0.0])
    e2 = np.cross(n_f, e1)
    axes = np.stack([e1, e2, n_f])
    t_box = _ray_box_frame(np.zeros(3), d, hit0, axes,
                           np.array([-0.15, -0.15, 0.0]), np.array([0.15, 0.15, 0.3]))
    t = np.minimum(t_floor, t_box)
    z = t * d[:, 2]
    z = z + rng.normal(0.0, 0.002, size=z.shape)
    pts = (d * z[:, None]).reshape(M, N, 3).astype(np.float32)
    _nan_uniform(pts, int(round(0.05 * M * N)), rng)
    return pts


def _blob_holes(M, N, target, rng):
    """Random 4-connected blobs of U{5..20} pixels until exactly `target`."""
    mask = np.zeros((M, N), dtype=bool)
    total = 0
    while total < target:
        size = min(int(rng.integers(5, 21)), target - total)
        while True:
            r0, c0 = int(rng.integers(0, M)), int(rng.integers(0, N))
            if not mask[r0, c0]:
                break
        blob = [(r0, c0)]
        mask[r0, c0] = True
        frontier = [(r0, c0)]
        while len(blob) < size and frontier:
            i = int(rng.integers(0, len(frontier)))
            r, c = frontier[i]
            nbrs = [(r + 1, c), (r - 1, c), (r, c + 1), (r, c - 1)]
            nbrs = [(a, b) for a, b in nbrs if 0 <= a < M and 0 <= b < N and not mask[a, b]]
            if not nbrs:
                frontier[i] = frontier[-1]
                frontier.pop()
                continue
            a, b = nbrs[int(rng.integers(0, len(nbrs)))]
            mask[a, b] = True
            blob.append((a, b))
            frontier.append((a, b))
        total += len(blob)
    return mask


def _rgbd_pose(rng):
    """Room corner and camera pose of the 480x640 scene (the first draws of its
    generator): wall distances wx, wy, yaw and the camera axes r, dn, f in the
    room frame (z up, floor at z = 0, walls x = wx and y = wy)."""
    wx, wy = rng.uniform(2.2, 3.8, size=2)
    yaw = math.atan2(wy, wx) + rng.uniform(-math.radians(5), math.radians(5))
    pitch = math.radians(20.0)
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), -math.sin(pitch)])
    r = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    dn = np.cross(f, r)
    return wx, wy, yaw, r, dn, f


def _rgbd(seed: int) -> np.ndarray:
    k = KINDS["rgbd"]
    M, N = k.M, k.N
    rng = np.random.default_rng(seed)
    fx = fy = 525.0
    cx, cy = 319.5, 239.5
    d_cam = _pinhole_dirs(M, N, fx, fy, cx, cy)
    wx, wy, yaw, r, dn, f = _rgbd_pose(rng)
    O = np.array([0.0, 0.0, 1.2])
    d = d_cam[:, :1] * r + d_cam[:, 1:2] * dn + d_cam[:, 2:3] * f
    inf = np.inf
    with np.errstate(divide="ignore", invalid="ignore"):
        t_floor = np.where(d[:, 2] < 0, -O[2] / d[:, 2], inf)
        t_wx = np.where(d[:, 0] > 0, (wx - O[0]) / d[:, 0], inf)
        t_wy = np.where(d[:, 1] > 0, (wy - O[1]) / d[:, 1], inf)
    t = np.minimum(np.minimum(t_floor, t_wx), t_wy)
    placed = 0
    while placed < 6:
        sides = rng.uniform(0.1, 0.5, size=3)
        rho = rng.uniform(1.2, 2.8)
        phi = yaw + rng.uniform(-math.radians(25), math.radians(25))
        cxy = np.array([rho * math.cos(phi), rho * math.sin(phi)])
        if cxy[0] > wx - 0.4 or cxy[1] > wy - 0.4:
            continue
        center = np.array([cxy[0], cxy[1], sides[2] / 2.0])
        t = np.minimum(t, _ray_box(O, d, center, rng.uniform(0, math.pi), sides / 2.0))
        placed += 1
    z = t * d_cam[:, 2]
    z = z + rng.normal(0.0, 1.0, size=z.shape) * 0.0012 * z * z
    pts = (d_cam * z[:, None]).reshape(M, N, 3).astype(np.float32)
    mask = _blob_holes(M, N, int(round(0.08 * M * N)), rng)
    pts[mask] = np.nan
    return pts


def _lidar(seed: int, M: int, N: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    elev = np.radians(3.0 - 28.0 * np.arange(M) / (M - 1))
    azim = 2.0 * np.pi * np.arange(N) / N
    E, A = np.meshgrid(elev, azim, indexing="ij")
    d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1).reshape(-1, 3)
    O = np.zeros(3)
    h, curb_y, curb_h = 1.73, 4.0, 0.15
    inf = np.inf
    with np.errstate(divide="ignore", invalid="ignore"):
        t_road = np.where(d[:, 2] < 0, -h / d[:, 2], inf)
        y_road = t_road * d[:, 1]
        t_road = np.where(np.abs(y_road) <= curb_y, t_road, inf)
        t_walk = np.where(d[:, 2] < 0, -(h - curb_h) / d[:, 2], inf)
        y_walk = t_walk * d[:, 1]
        t_walk = np.where(np.abs(y_walk) >= curb_y, t_walk, inf)
        t_curb = np.where(d[:, 1] != 0, curb_y / np.abs(d[:, 1]), inf)
        z_curb = t_curb * d[:, 2]
        t_curb = np.where((z_curb >= -h) & (z_curb <= -(h - curb_h)), t_curb, inf)
    t = np.minimum(np.minimum(t_road, t_walk), t_curb)
    placed = 0
    half = np.array([2.25, 0.9, 0.75])
    while placed < 10:
        rad = 40.0 * math.sqrt(rng.uniform())
        th = rng.uniform(0, 2 * math.pi)
        if rad < 3.0 + 2.5:
            continue
        center = np.array([rad * math.cos(th), rad * math.sin(th), -h + 0.75])
        t = np.minimum(t, _ray_box(O, d, center, rng.uniform(0, math.pi), half))
        placed += 1
    valid = t <= 120.0
    rng_t = np.where(valid, t, 0.0) + rng.normal(0.0, 0.02, size=t.shape)
    pts = (d * rng_t[:, None]).astype(np.float32)
    pts[~valid] = np.nan
    vidx = np.flatnonzero(valid)
    drop = rng.choice(vidx, size=min(int(round(0.10 * M * N)), vidx.size), replace=False)
    pts[drop] = np.nan
    return pts.reshape(M, N, 3)


def make_frame(kind: str, seed: int) -> np.ndarray:
    """One synthetic frame of the given kind, float32 [M, N, 3], NaN = invalid."""
    if kind == "rgbd_small":
        return _rgbd_small(seed)
    if kind == "rgbd":
        return _rgbd(seed)
    if kind == "lidar":
        return _lidar(seed, 64, 1024)
    if kind == "lidar128":
        return _lidar(seed, 128, 2048)
    raise ValueError(f"unknown frame kind {kind!r}")


def scene_planes(kind: str, seed: int) -> np.ndarray:
    """Unit normals of the large planes of frame (kind, seed), float32 [l, 3],
    in the frame's own coordinates: the dominant plane normals a plane
    detector would report for it, given as known inputs.

    120x160: the floor and the cube face turned toward the camera.  480x640:
    the floor and the two walls.  LiDAR: the road (and sidewalk tops) and the
    two curb faces.  Each normal is oriented the way the frame's triangles
    wind: toward the sensor for the pinhole frames and away from it for the
    LiDAR frames, whose azimuth runs to the left as seen from the sensor and
    so mirrors the image grid."""
    if kind == "rgbd_small":
        t = _SMALL_TILT
        n_f = np.array([0.0, -math.sin(t), -math.cos(t)])
        e2 = np.cross(n_f, np.array([1.0, 0.0, 0.0]))
        planes = np.stack([n_f, -e2])
    elif kind == "rgbd":
        _, _, _, r, dn, f = _rgbd_pose(np.random.default_rng(seed))
        world = np.array([[0.0, 0.0, 1.0], [-1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
        planes = np.stack([world @ r, world @ dn, world @ f], axis=1)
    elif kind in ("lidar", "lidar128"):
        planes = -np.array([[0.0, 0.0, 1.0], [0.0, -1.0, 0.0], [0.0, 1.0, 0.0]])
    else:
        raise ValueError(f"unknown frame kind {kind!r}")
    planes = planes / np.linalg.norm(planes, axis=1, keepdims=True)
    return planes.astype(np.float32)


def config_frame(config: int, frame: int = 0) -> tuple[np.ndarray, FrameKind]:
    """Frame `frame` of single-frame workload `config` (0: 120x160 RGBD,
    1: 480x640 RGBD, 2: 64x1024 LiDAR); seed = 1000 * config + frame."""
    kind = CONFIG_KIND[config]
    return make_frame(kind, 1000 * config + frame), KINDS[kind]


def batch_mix() -> list[tuple[str, int]]:
    """The 64-frame mixed batch: 16x 120x160, 24x 480x640, 16x 64x1024 and
    8x 128x2048, as (kind, seed) with seed = 3000 + position."""
    kinds = ["rgbd_small"] * 16 + ["rgbd"] * 24 + ["lidar"] * 16 + ["lidar128"] * 8
    return [(k, 3000 + i) for i, k in enumerate(kinds)]


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int = 4000,
                     mix=(("rgbd", 0.4), ("lidar", 0.3), ("lidar128", 0.2), ("rgbd_small", 0.1))):
    """Arrival times (s) and frame kinds of a Poisson stream: exponential gaps
    at `rate_hz`, kinds drawn with the given probabilities."""
    rng = np.random.default_rng(seed)
    times, kinds = [], []
    names = [m[0] for m in mix]
    probs = np.array([m[1] for m in mix], dtype=np.float64)
    probs = probs / probs.sum()
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        times.append(t)
        kinds.append(names[int(rng.choice(len(names), p=probs))])
    return np.array(times), kinds


def random_grid(M: int, N: int, seed: int, nan_frac: float = 0.1,
                noise: float = 0.01) -> np.ndarray:
    """Small test grid: a gently curved surface seen from the origin, with
    Gaussian noise and a random fraction of NaN pixels.  float32 [M, N, 3]."""
    rng = np.random.default_rng(seed)
    v, u = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(M, dtype=np.float64))
    x = 0.05 * (v - N / 2.0)
    y = 0.05 * (u - M / 2.0)
    z = 2.0 + 0.3 * np.sin(0.4 * v) * np.cos(0.3 * u) + rng.normal(0.0, noise, size=u.shape)
    pts = np.stack([x, y, z], axis=-1) + rng.normal(0.0, noise, size=(M, N, 3))
    pts = pts.astype(np.float32)
    if nan_frac > 0:
        m = rng.random((M, N)) < nan_frac
        pts[m] = np.nan
    return pts
