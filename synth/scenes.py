"""Analytic scenes, camera trajectories and depth frames (float64 numpy, seeded).

Conventions (shared with the library's public header):
  * metres; camera frame x right, y down, z forward; pinhole, no distortion;
  * pixel (u, v) has its centre at integer coordinates, its ray in the camera frame
    is ((u - cx) / fx, (v - cy) / fy, 1);
  * a pose T_wc is a row-major 4x4 float64 camera-to-world transform;
  * a depth frame is float32 [H, W], the camera-z of the first surface hit,
    0 where the sensor has no measurement.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# workloads: image geometry, scene parameters and stream recipe per named setup
# ---------------------------------------------------------------------------
WORKLOADS = {
    # 10 frames 160x120; sphere r=0.3 m at 1.2 m on a plane at 1.8 m; 10-degree arc
    "tiny": dict(width=160, height=120, fx=140.0, fy=140.0, cx=80.0, cy=60.0,
                 n_frames=10, voxel_size=0.01, mu=0.04, max_w=100,
                 n_buckets=2 ** 14, n_excess=2 ** 12, seed=0),
    # 300 frames VGA through a 4x4x3 m room with 20 boxes and 10 spheres
    "vga": dict(width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5,
                n_frames=300, voxel_size=0.005, mu=0.02, max_w=100,
                n_buckets=2 ** 20, n_excess=2 ** 17, seed=1),
    # 1000 frames VGA through a 20x20x3 m grid of 5x5 m rooms with 200 boxes
    "large": dict(width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5,
                  n_frames=1000, voxel_size=0.004, mu=0.016, max_w=100,
                  n_buckets=2 ** 22, n_excess=2 ** 19, seed=3),
    # rooms in the "vga" style, 100 frames each, for (5-frame, 100-frame) pairs
    "room": dict(width=640, height=480, fx=525.0, fy=525.0, cx=319.5, cy=239.5,
                 n_frames=100, voxel_size=0.005, mu=0.02, max_w=100,
                 n_buckets=2 ** 20, n_excess=2 ** 17, seed=1000),
}

SENSOR_MAX_DEPTH = 4.0      # metres; farther returns are dropped
NOISE_K = 0.0012            # sigma = NOISE_K * z^2 (metres)


def workload_params(name: str) -> dict:
    return dict(WORKLOADS[name])


# ---------------------------------------------------------------------------
# scene description
# ---------------------------------------------------------------------------
@dataclass
class Scene:
    """Union of solids. `room` is an interior box the camera lives in (its walls
    are surfaces seen from inside); `boxes` are solid axis-aligned boxes [n, 2, 3]
    (lo, hi); `spheres` are [n, 4] (centre, radius); `planes` are [n, 4] (unit
    normal pointing to free space, offset h) meaning the surface n.x = h with the
    solid on the side n.x < h."""
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 2, 3)))
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    planes: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    room: np.ndarray | None = None

    def signed_distance(self, p: np.ndarray) -> np.ndarray:
        """Euclidean distance to the nearest surface, positive in free space,
        for points p [..., 3] (exact outside all solids)."""
        p = np.asarray(p, dtype=np.float64)
        sd = np.full(p.shape[:-1], np.inf)
        if self.room is not None:
            lo, hi = self.room
            sd = np.minimum(sd, np.min(np.concatenate([p - lo, hi - p], axis=-1), axis=-1))
        for lo, hi in self.boxes:
            q = np.maximum(lo - p, p - hi)
            outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
            inside = np.minimum(np.max(q, axis=-1), 0.0)
            sd = np.minimum(sd, outside + inside)
        for c in self.spheres:
            sd = np.minimum(sd, np.linalg.norm(p - c[:3], axis=-1) - c[3])
        for pl in self.planes:
            sd = np.minimum(sd, p @ pl[:3] - pl[3])
        return sd

    def clearance(self, p: np.ndarray) -> float:
        return float(self.signed_distance(np.asarray(p, dtype=np.float64)[None])[0])


@dataclass
class Stream:
    name: str
    depth: np.ndarray          # [F, H, W] float32, metres, 0 = invalid
    T_wc: np.ndarray           # [F, 4, 4] float64 camera -> world
    intrinsics: tuple          # (fx, fy, cx, cy)
    width: int
    height: int
    params: dict               # voxel_size, mu, max_w, n_buckets, n_excess
    scene: Scene
    seed: int
    noise: bool

    @property
    def n_frames(self) -> int:
        return self.depth.shape[0]


# ---------------------------------------------------------------------------
# poses
# ---------------------------------------------------------------------------
def pose_look_at(eye, target, up) -> np.ndarray:
    """Camera-to-world pose with the camera at `eye` looking at `target`;
    `up` is the world direction that should appear upward in the image."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = x, y, z, eye
    return T


def _rot(axis: int, a: float) -> np.ndarray:
    c, s = np.cos(a), np.sin(a)
    R = np.eye(3)
    i, j = [(1, 2), (2, 0), (0, 1)][axis]
    R[i, i], R[i, j], R[j, i], R[j, j] = c, -s, s, c
    return R


# y-up world; camera looking along -z with image "up" = +y
_R0 = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, -1.0]])


def _pose_from_angles(pos, yaw, pitch, roll) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = _rot(1, yaw) @ _R0 @ _rot(0, pitch) @ _rot(2, roll)
    T[:3, 3] = pos
    return T


# ---------------------------------------------------------------------------
# rendering
# ---------------------------------------------------------------------------
def _aabb_distance(p, lo, hi):
    return np.linalg.norm(np.maximum(np.maximum(lo - p, p - hi), 0.0), axis=-1)


def _rect(pts_w, T_wc, intrinsics, width, height):
    """Pixel rectangle [v0:v1, u0:u1] covering the projection of the points
    pts_w [n, 3]; the full image if any point is at or behind the camera plane."""
    fx, fy, cx, cy = intrinsics
    R, o = T_wc[:3, :3], T_wc[:3, 3]
    pc = (pts_w - o) @ R
    if np.any(pc[:, 2] <= 1e-6):
        return 0, height, 0, width
    u = fx * pc[:, 0] / pc[:, 2] + cx
    v = fy * pc[:, 1] / pc[:, 2] + cy
    u0, u1 = int(np.floor(u.min())) - 1, int(np.ceil(u.max())) + 2
    v0, v1 = int(np.floor(v.min())) - 1, int(np.ceil(v.max())) + 2
    return max(v0, 0), min(v1, height), max(u0, 0), min(u1, width)


def _corners(lo, hi):
    return np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1])
                     for z in (lo[2], hi[2])])


def render_depth(scene: Scene, intrinsics, width: int, height: int, T_wc: np.ndarray,
                 cull: float = np.inf) -> np.ndarray:
    """Exact camera-z of the first hit per pixel (float64 [H, W], inf = no hit).
    Primitives farther than `cull` metres from the camera are skipped (their hits
    would be dropped by the sensor range anyway); each solid is only tested on the
    pixels its bounding box projects to."""
    fx, fy, cx, cy = intrinsics
    xs = (np.arange(width, dtype=np.float64) - cx) / fx
    ys = (np.arange(height, dtype=np.float64) - cy) / fy
    R, o = T_wc[:3, :3], T_wc[:3, 3]
    # world direction with camera-z = 1, one [H, W] array per axis
    d = [R[a, 0] * xs[None, :] + R[a, 1] * ys[:, None] + R[a, 2] for a in range(3)]
    t = np.full((height, width), np.inf)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        inv = [1.0 / d[a] for a in range(3)]
        if scene.room is not None:
            lo, hi = scene.room
            for a in range(3):
                t = np.minimum(t, np.maximum((lo[a] - o[a]) * inv[a], (hi[a] - o[a]) * inv[a]))
        for lo, hi in scene.boxes:
            if _aabb_distance(o, lo, hi) > cull:
                continue
            v0, v1, u0, u1 = _rect(_corners(lo, hi), T_wc, intrinsics, width, height)
            if v0 >= v1 or u0 >= u1:
                continue
            tn = tf = None
            for a in range(3):
                ia = inv[a][v0:v1, u0:u1]
                t1, t2 = (lo[a] - o[a]) * ia, (hi[a] - o[a]) * ia
                mn, mx = np.minimum(t1, t2), np.maximum(t1, t2)
                tn = mn if tn is None else np.maximum(tn, mn)
                tf = mx if tf is None else np.minimum(tf, mx)
            ts = t[v0:v1, u0:u1]
            hit = (tn <= tf) & (tn > 0) & (tn < ts)
            ts[hit] = tn[hit]
        for c in scene.spheres:
            if np.linalg.norm(o - c[:3]) - c[3] > cull:
                continue
            r = c[3]
            v0, v1, u0, u1 = _rect(_corners(c[:3] - r, c[:3] + r), T_wc, intrinsics, width, height)
            if v0 >= v1 or u0 >= u1:
                continue
            oc = o - c[:3]
            ds = [d[a][v0:v1, u0:u1] for a in range(3)]
            a2 = ds[0] * ds[0] + ds[1] * ds[1] + ds[2] * ds[2]
            b = ds[0] * oc[0] + ds[1] * oc[1] + ds[2] * oc[2]
            cc = oc @ oc - r * r
            disc = b * b - a2 * cc
            ok = disc >= 0
            th = (-b - np.sqrt(np.where(ok, disc, 0.0))) / a2
            ts = t[v0:v1, u0:u1]
            hit = ok & (th > 0) & (th < ts)
            ts[hit] = th[hit]
        for pl in scene.planes:
            den = d[0] * pl[0] + d[1] * pl[1] + d[2] * pl[2]
            th = (pl[3] - o @ pl[:3]) / den
            hit = (den < 0) & (th > 0) & (th < t)
            t[hit] = th[hit]
    return t


def render_plane_maps(planes, intrinsics, width: int, height: int, T_wc: np.ndarray):
    """Reference maps of a scene of planes (rows n_x, n_y, n_z, c: the plane
    n . x = c, hit from the side its unit normal faces): camera-z of the first hit
    per pixel (float64 [H, W], 0 = no hit), and the hit's world point and normal
    as float32 [H, W, 4] with w = 1 (all zero on a miss)."""
    planes = np.asarray(planes, np.float64)
    fx, fy, cx, cy = intrinsics
    xs = (np.arange(width, dtype=np.float64) - cx) / fx
    ys = (np.arange(height, dtype=np.float64) - cy) / fy
    R, o = T_wc[:3, :3], T_wc[:3, 3]
    d = np.stack([R[a, 0] * xs[None, :] + R[a, 1] * ys[:, None] + R[a, 2] for a in range(3)], -1)
    t = np.full((height, width), np.inf)
    idx = np.full((height, width), -1)
    with np.errstate(divide="ignore", invalid="ignore"):
        for i, pl in enumerate(planes):
            den = d @ pl[:3]
            th = (pl[3] - o @ pl[:3]) / den
            hit = (den < 0) & (th > 0) & (th < t)
            t[hit] = th[hit]
            idx[hit] = i
    hit = idx >= 0
    depth = np.where(hit, t, 0.0)   # camera z: the direction has camera-z 1
    V = np.zeros((height, width, 4), np.float32)
    N = np.zeros((height, width, 4), np.float32)
    P = o + d * np.where(hit, t, 0.0)[..., None]
    V[..., :3] = np.where(hit[..., None], P, 0.0)
    V[..., 3] = hit
    N[..., :3] = np.where(hit[..., None], planes[np.maximum(idx, 0), :3], 0.0)
    N[..., 3] = hit
    return depth, V, N


def _sensor(z: np.ndarray, rng, noise: bool, invalid_frac: float) -> np.ndarray:
    z = z.copy()
    if noise:
        z = z + rng.standard_normal(z.shape) * (NOISE_K * z * z)
    bad = ~np.isfinite(z) | (z <= 0) | (z > SENSOR_MAX_DEPTH)
    if invalid_frac > 0:
        bad |= rng.random(z.shape) < invalid_frac
    z[bad] = 0.0
    return z.astype(np.float32)


# ---------------------------------------------------------------------------
# scene + trajectory recipes
# ---------------------------------------------------------------------------
def _tiny_scene():
    return Scene(spheres=np.array([[0.0, 0.0, 1.2, 0.3]]),
                 planes=np.array([[0.0, 0.0, -1.0, -1.8]]))


def _tiny_poses(n):
    c = np.array([0.0, 0.0, 1.2])
    poses = []
    for a in np.deg2rad(np.linspace(-5.0, 5.0, n)):
        eye = c + 1.2 * np.array([np.sin(a), 0.0, -np.cos(a)])
        poses.append(pose_look_at(eye, c, up=(0.0, -1.0, 0.0)))
    return np.stack(poses)


def _room_scene(rng, size=(4.0, 3.0, 4.0), n_boxes=20, n_spheres=10, keep_free=None,
                keep_r=0.8):
    lo, hi = np.zeros(3), np.array(size, np.float64)
    boxes, spheres = [], []
    free = keep_free if keep_free is not None else (lo + hi) / 2

    def clear_of_start(sd_fn):
        return sd_fn(free) > keep_r

    while len(boxes) < n_boxes:
        s = rng.uniform(0.1, 0.8, 3)
        p = np.array([rng.uniform(0, hi[0] - s[0]), 0.0, rng.uniform(0, hi[2] - s[2])])
        b = np.stack([p, p + s])
        if clear_of_start(lambda q: _aabb_distance(q, b[0], b[1])):
            boxes.append(b)
    while len(spheres) < n_spheres:
        r = rng.uniform(0.1, 0.8) / 2
        c = rng.uniform(lo + r, hi - r)
        if clear_of_start(lambda q: np.linalg.norm(q - c) - r):
            spheres.append(np.append(c, r))
    return Scene(boxes=np.array(boxes), spheres=np.array(spheres), room=np.stack([lo, hi]))


def _walk_poses(scene: Scene, rng, n, start, step=0.01, dang=np.deg2rad(1.0),
                clearance=0.3):
    pos = np.array(start, np.float64)
    vel = rng.standard_normal(3)
    vel /= np.linalg.norm(vel)
    ang = np.array([rng.uniform(0, 2 * np.pi), 0.0, 0.0])
    angv = np.zeros(3)
    poses = []
    for _ in range(n):
        poses.append(_pose_from_angles(pos, *ang))
        vel = 0.9 * vel + 0.1 * rng.standard_normal(3)
        vel /= np.linalg.norm(vel)
        new = pos + step * vel
        if scene.clearance(new) < clearance:
            vel = -vel
        else:
            pos = new
        angv = 0.9 * angv + 0.1 * rng.standard_normal(3)
        a = angv / max(np.abs(angv).max(), 1e-12) * dang
        ang = ang + a
        ang[1] = np.clip(ang[1], -np.deg2rad(30), np.deg2rad(30))
        ang[2] = np.clip(ang[2], -np.deg2rad(10), np.deg2rad(10))
    return np.stack(poses)


def _grid_scene(rng, n_boxes=200):
    """4x4 grid of 5x5 m rooms in [0,20]x[0,3]x[0,20]; 0.1 m interior walls with a
    1 m doorway in the middle of every wall segment."""
    H, half_t = 3.0, 0.05
    walls = []
    for k in (5.0, 10.0, 15.0):
        for j in range(4):
            z0, z1 = 5.0 * j, 5.0 * j + 5.0
            for a, b in ((z0, z0 + 2.0), (z0 + 3.0, z1)):
                walls.append(np.array([[k - half_t, 0.0, a], [k + half_t, H, b]]))   # x = k
                walls.append(np.array([[a, 0.0, k - half_t], [b, H, k + half_t]]))   # z = k
    path = _grid_path()
    boxes = []
    while len(boxes) < n_boxes:
        s = rng.uniform(0.1, 0.8, 3)
        p = np.array([rng.uniform(0, 20 - s[0]), 0.0, rng.uniform(0, 20 - s[2])])
        b = np.stack([p, p + s])
        seg_d = _polyline_box_distance(path, b[0], b[1])
        if seg_d > 0.7:
            boxes.append(b)
    room = np.array([[0.0, 0.0, 0.0], [20.0, H, 20.0]])
    return Scene(boxes=np.concatenate([np.array(walls), np.array(boxes)]), room=room), path


def _grid_path():
    """Room centres in boustrophedon order, joined through the doorways."""
    pts = []
    for j in range(4):
        cols = range(4) if j % 2 == 0 else range(3, -1, -1)
        for i in cols:
            pts.append((2.5 + 5 * i, 1.5, 2.5 + 5 * j))
    out = [np.array(pts[0])]
    for a, b in zip(pts[:-1], pts[1:]):
        a, b = np.array(a), np.array(b)
        out.append((a + b) / 2)   # doorway centre
        out.append(b)
    return np.array(out)


def _polyline_box_distance(path, lo, hi, n=20):
    best = np.inf
    for a, b in zip(path[:-1], path[1:]):
        s = np.linspace(0, 1, n)[:, None]
        q = a + s * (b - a)
        best = min(best, float(_aabb_distance(q, lo, hi).min()))
    return best


def _path_poses(path, rng, n, step=0.06, dang=np.deg2rad(1.0)):
    seg = np.linalg.norm(np.diff(path, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    poses = []
    jit = np.zeros(3)
    for f in range(n):
        s = min(f * step, cum[-1] - 1e-9)
        k = int(np.searchsorted(cum, s, side="right") - 1)
        k = min(k, len(seg) - 1)
        a = (s - cum[k]) / seg[k]
        pos = path[k] + a * (path[k + 1] - path[k])
        dirv = path[k + 1] - path[k]
        yaw = np.arctan2(-dirv[0], -dirv[2])      # camera looks along -z at yaw 0
        jit = 0.9 * jit + 0.1 * rng.standard_normal(3)
        j = jit / max(np.abs(jit).max(), 1e-12) * dang * 5
        poses.append(_pose_from_angles(pos, yaw + j[0], 0.2 * j[1], 0.1 * j[2]))
    return np.stack(poses)


_STREAM_CACHE: dict = {}


# the colour of a surface point: three smooth waves in world space, one per
# channel (wavelengths 0.3-0.5 m), mid grey +- 110
_CLR_DIR = np.array([[2.3, 0.7, -1.1], [-0.9, 2.8, 0.6], [1.2, -1.4, 2.5]])
_CLR_PHASE = np.array([0.3, 1.9, 4.1])


def colour_frames(stream: Stream, frames=None, seed: int = 17) -> np.ndarray:
    """Registered colour images (same camera as the depth): uint8 [n, H, W, 4]
    (R, G, B, 0), the colour of the world point each valid depth pixel sees, with
    sensor noise (sigma 1.5 levels); black where the depth is invalid."""
    frames = range(stream.n_frames) if frames is None else frames
    rng = np.random.default_rng(seed)
    fx, fy, cx, cy = stream.intrinsics
    W, H = stream.width, stream.height
    xs = (np.arange(W, dtype=np.float64) - cx) / fx
    ys = (np.arange(H, dtype=np.float64) - cy) / fy
    out = np.zeros((len(frames), H, W, 4), np.uint8)
    for i, f in enumerate(frames):
        d = stream.depth[f].astype(np.float64)
        ok = np.isfinite(d) & (d > 0)
        dd = np.where(ok, d, 0.0)
        R, o = stream.T_wc[f][:3, :3], stream.T_wc[f][:3, 3]
        q = np.stack([xs[None, :] * dd, ys[:, None] * dd, dd], -1)
        P = q @ R.T + o
        c = 128.0 + 110.0 * np.sin(P @ _CLR_DIR.T * (2.0 * np.pi / 1.6) + _CLR_PHASE)
        c = np.clip(np.rint(c + rng.standard_normal(c.shape) * 1.5), 0, 255)
        out[i, ..., :3] = np.where(ok[..., None], c, 0).astype(np.uint8)
    return out


def make_stream(name: str, n_frames: int | None = None, seed: int | None = None,
                noise: bool = True, cache: bool = True) -> Stream:
    """Seeded synthetic stream for a named workload ("tiny", "vga", "large", "room").
    `noise=False` gives exact depth (used by the closed-form checks)."""
    p = workload_params(name)
    seed = p["seed"] if seed is None else seed
    n = p["n_frames"] if n_frames is None else n_frames
    key = (name, n, seed, noise)
    if cache and key in _STREAM_CACHE:
        return _STREAM_CACHE[key]
    rng = np.random.default_rng(seed)
    K = (p["fx"], p["fy"], p["cx"], p["cy"])
    W, H = p["width"], p["height"]
    invalid = 0.0
    if name == "tiny":
        scene, poses = _tiny_scene(), _tiny_poses(n)
    elif name in ("vga", "room"):
        scene = _room_scene(rng)
        poses = _walk_poses(scene, rng, n, start=(2.0, 1.5, 2.0))
        invalid = 0.05 if noise else 0.0
    elif name == "large":
        scene, path = _grid_scene(rng)
        poses = _path_poses(path, rng, n)
        invalid = 0.05 if noise else 0.0
    else:
        raise KeyError(name)
    cull = SENSOR_MAX_DEPTH + 0.5 if name != "tiny" else np.inf
    depth = np.empty((n, H, W), np.float32)
    # rendering is independent per frame (numpy releases the GIL); the sensor
    # model draws from the one seeded generator in frame order afterwards
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        exact = list(ex.map(lambda f: render_depth(scene, K, W, H, poses[f], cull=cull), range(n)))
    for f in range(n):
        depth[f] = _sensor(exact[f], rng, noise, invalid)
        exact[f] = None
    st = Stream(name=name, depth=depth, T_wc=poses, intrinsics=K, width=W, height=H,
                params={k: p[k] for k in ("voxel_size", "mu", "max_w", "n_buckets", "n_excess")},
                scene=scene, seed=seed, noise=noise)
    if cache:
        _STREAM_CACHE[key] = st
    return st
