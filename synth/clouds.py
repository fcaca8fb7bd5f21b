"""Seeded scene generators.

Every generator takes an integer seed and returns float32 clouds in metres.
Randomness: ``numpy.random.Generator(PCG64)`` streams obtained from
``SeedSequence(seed).spawn(3)``: stream 0 builds the data, stream 1 draws the
initial particles, stream 2 draws the minibatch schedule.

Pose convention of the returned ground truth ``theta_true`` (six-vector
x, y, z, roll, pitch, yaw): it maps source points onto the reference,
``r = Rz(yaw) Ry(pitch) Rx(roll) s + (x, y, z)``; the rotation is produced and
decomposed by scipy's ``Rotation`` with the intrinsic ``"ZYX"`` sequence.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation


@dataclass
class Pair:
    name: str
    src: np.ndarray          # float32 (N, 3)
    ref: np.ndarray          # float32 (M, 3)
    theta_true: np.ndarray   # float64 (6,), maps src onto ref
    meta: dict = field(default_factory=dict)


def rng_streams(seed: int):
    """Three independent PCG64 generators: (data, init, minibatch)."""
    ss = np.random.SeedSequence(int(seed))
    return tuple(np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3))


# ---------------------------------------------------------------------------
# rigid motion helpers (scipy only)
# ---------------------------------------------------------------------------

def _random_rigid(rng, half_t: float, half_deg: float):
    t = rng.uniform(-half_t, half_t, size=3)
    ypr = np.deg2rad(rng.uniform(-half_deg, half_deg, size=3))  # yaw, pitch, roll
    rot = Rotation.from_euler("ZYX", ypr)
    return rot, t


def _theta_of_inverse(rot: Rotation, t: np.ndarray) -> np.ndarray:
    """Pose (x,y,z,roll,pitch,yaw) of the inverse of ``p -> rot p + t``."""
    inv = rot.inv()
    trans = -inv.apply(t)
    yaw, pitch, roll = inv.as_euler("ZYX")
    return np.array([trans[0], trans[1], trans[2], roll, pitch, yaw], dtype=np.float64)


def _move_source(rng, pts, half_t=0.1, half_deg=15.0):
    """Move ``pts`` by a seeded rigid transform; return moved points and the
    pose that maps them back (the ground truth for registration)."""
    rot, t = _random_rigid(rng, half_t, half_deg)
    moved = rot.apply(pts.astype(np.float64)) + t
    return moved, _theta_of_inverse(rot, t)


# ---------------------------------------------------------------------------
# cuboid (small RGB-D object stand-in)
# ---------------------------------------------------------------------------

def _cuboid_surface(rng, n: int, dims=(0.30, 0.20, 0.10)) -> np.ndarray:
    """Points uniform on the surface of an axis-aligned box centred at 0;
    faces chosen in proportion to their area."""
    a, b, c = dims
    areas = np.array([b * c, b * c, a * c, a * c, a * b, a * b])
    face = rng.choice(6, size=n, p=areas / areas.sum())
    u = rng.uniform(-0.5, 0.5, size=n)
    v = rng.uniform(-0.5, 0.5, size=n)
    p = np.empty((n, 3))
    half = np.array(dims) / 2
    for f in range(6):
        sel = face == f
        axis = f // 2                       # 0: x faces, 1: y faces, 2: z faces
        sign = 1.0 if f % 2 == 0 else -1.0
        others = [d for d in range(3) if d != axis]
        p[sel, axis] = sign * half[axis]
        p[sel, others[0]] = u[sel] * dims[others[0]]
        p[sel, others[1]] = v[sel] * dims[others[1]]
    return p


def cuboid_pair(seed: int, n_src: int = 500, n_ref: int = 2000,
                noise: float = 0.002, dims=(0.30, 0.20, 0.10)) -> Pair:
    """Box 0.30 x 0.20 x 0.10 m. Reference: ``n_ref`` surface samples plus iid
    N(0, noise^2) per coordinate. Source: ``n_src`` fresh samples with the same
    noise, moved by translation U(+-0.1 m) and roll/pitch/yaw U(+-15 deg)."""
    rng, _, _ = rng_streams(seed)
    ref = _cuboid_surface(rng, n_ref, dims) + rng.normal(0, noise, (n_ref, 3))
    src0 = _cuboid_surface(rng, n_src, dims) + rng.normal(0, noise, (n_src, 3))
    src, theta = _move_source(rng, src0)
    return Pair("cuboid", src.astype(np.float32), ref.astype(np.float32), theta,
                {"seed": seed, "dims": dims, "noise": noise})


# ---------------------------------------------------------------------------
# ray casting against planes, boxes and vertical cylinders
# ---------------------------------------------------------------------------

def _hit_plane_z0(o, d, extent=None):
    with np.errstate(divide="ignore", invalid="ignore"):
        t = -o[:, 2] / d[:, 2]
    t = np.where((t > 1e-9) & np.isfinite(t), t, np.inf)
    if extent is not None:
        p = o + np.where(np.isfinite(t), t, 0)[:, None] * d
        inside = (np.abs(p[:, 0]) <= extent) & (np.abs(p[:, 1]) <= extent)
        t = np.where(inside, t, np.inf)
    return t


def _hit_box(o, d, lo, hi):
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (lo - o) * inv
        t1 = (hi - o) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=1)
    ok = (tmax >= tmin) & (tmin > 1e-9)
    return np.where(ok, tmin, np.inf)


def _hit_cylinder(o, d, cx, cy, r, z0, z1):
    """Vertical cylinder side wall plus top cap."""
    ox, oy = o[:, 0] - cx, o[:, 1] - cy
    a = d[:, 0] ** 2 + d[:, 1] ** 2
    b = 2 * (ox * d[:, 0] + oy * d[:, 1])
    c = ox ** 2 + oy ** 2 - r * r
    disc = b * b - 4 * a * c
    with np.errstate(divide="ignore", invalid="ignore"):
        sq = np.sqrt(np.maximum(disc, 0))
        t_side = (-b - sq) / (2 * a)
    z = o[:, 2] + t_side * d[:, 2]
    side_ok = (disc >= 0) & (a > 1e-12) & (t_side > 1e-9) & (z >= z0) & (z <= z1)
    t_side = np.where(side_ok, t_side, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        t_cap = (z1 - o[:, 2]) / d[:, 2]
    px = o[:, 0] + t_cap * d[:, 0] - cx
    py = o[:, 1] + t_cap * d[:, 1] - cy
    cap_ok = np.isfinite(t_cap) & (t_cap > 1e-9) & (px * px + py * py <= r * r)
    t_cap = np.where(cap_ok, t_cap, np.inf)
    return np.minimum(t_side, t_cap)


def _cast(o, d, prims, chunk=200_000):
    """Nearest hit distance along each ray over all primitives (inf = miss)."""
    out = np.full(len(d), np.inf)
    for s in range(0, len(d), chunk):
        oo = o[s:s + chunk] if o.ndim == 2 else np.broadcast_to(o, d[s:s + chunk].shape)
        dd = d[s:s + chunk]
        best = np.full(len(dd), np.inf)
        for kind, args in prims:
            if kind == "plane":
                t = _hit_plane_z0(oo, dd, *args)
            elif kind == "box":
                t = _hit_box(oo, dd, *args)
            else:
                t = _hit_cylinder(oo, dd, *args)
            best = np.minimum(best, t)
        out[s:s + chunk] = best
    return out


# ---------------------------------------------------------------------------
# Kinect-shaped tabletop
# ---------------------------------------------------------------------------

_KINECT_FOV = (np.deg2rad(57.0), np.deg2rad(43.0))


def _pinhole_rays(cam_pos, target, width=640, height=480):
    f = target - cam_pos
    f = f / np.linalg.norm(f)
    right = np.cross(f, [0.0, 0.0, 1.0])
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    tx = np.tan(_KINECT_FOV[0] / 2)
    ty = np.tan(_KINECT_FOV[1] / 2)
    xs = np.linspace(-tx, tx, width)
    ys = np.linspace(-ty, ty, height)
    gx, gy = np.meshgrid(xs, ys)
    d = f[None, :] + gx.reshape(-1, 1) * right[None, :] + gy.reshape(-1, 1) * down[None, :]
    dn = np.linalg.norm(d, axis=1, keepdims=True)
    return d / dn, (1.0 / dn[:, 0]), f   # unit rays, depth per unit range, axis


def _kinect_scene(rng):
    cyl = (rng.uniform(-0.2, 0.0), rng.uniform(-0.15, 0.15), 0.04, 0.0, 0.2)
    bx, by = rng.uniform(0.08, 0.25), rng.uniform(-0.15, 0.15)
    box_lo = np.array([bx - 0.06, by - 0.04, 0.0])
    box_hi = np.array([bx + 0.06, by + 0.04, 0.10])
    return [("plane", (0.5,)), ("cylinder", cyl), ("box", (box_lo, box_hi))]


def _kinect_view(rng, prims, cam_pos, target, noisy=True, res=(640, 480)):
    d, depth_per_t, _ = _pinhole_rays(cam_pos, target, *res)
    t = _cast(cam_pos, d, prims)
    z = t * depth_per_t
    keep = np.isfinite(t) & (z >= 0.5) & (z <= 1.5)
    t, z, d = t[keep], z[keep], d[keep]
    clean = cam_pos + t[:, None] * d
    if not noisy:
        return clean, None
    tn = t + rng.normal(0.0, 1.0, size=len(t)) * 0.0015 * z * z
    return clean, cam_pos + tn[:, None] * d


def kinect_pair(seed: int, n_src: int = 20000, n_ref: int = 20000,
                overlap: float = 0.70) -> Pair:
    """Tabletop: 1 x 1 m ground plane, a cylinder (r 0.04 m, h 0.2 m) and a
    0.12 x 0.08 x 0.10 m box, seen by a 640 x 480 pinhole camera with a
    57 x 43 deg field of view; depth kept in [0.5, 1.5] m, noise along the ray
    with sigma 0.0015 z^2. The second viewpoint is shifted sideways by a
    bisection until the overlap reaches ``overlap``: the smaller of the two
    fractions of one view's noise-free points lying within 1 cm of the other
    view's noise-free points. The source (second view) is then
    moved by a seeded rigid transform as for the cuboid."""
    rng, _, _ = rng_streams(seed)
    prims = _kinect_scene(rng)
    az = rng.uniform(0, 2 * np.pi)
    cam1 = np.array([0.95 * np.cos(az), 0.95 * np.sin(az), 0.55])
    target = np.array([0.0, 0.0, 0.05])
    clean1, noisy1 = _kinect_view(rng, prims, cam1, target)
    coarse1, _ = _kinect_view(rng, prims, cam1, target, noisy=False, res=(320, 240))
    tree = cKDTree(coarse1)
    fwd = target - cam1
    side = np.cross(fwd, [0.0, 0.0, 1.0])
    side /= np.linalg.norm(side)

    def frac(shift):
        c2, _ = _kinect_view(rng, prims, cam1 + shift * side, target + shift * side,
                             noisy=False, res=(320, 240))
        d21, _ = tree.query(c2, k=1)
        d12, _ = cKDTree(c2).query(coarse1, k=1)
        return min(float(np.mean(d21 <= 0.01)), float(np.mean(d12 <= 0.01))), c2

    lo, hi = 0.0, 0.8
    best_shift, best_err = 0.0, 1.0
    for _ in range(18):
        mid = 0.5 * (lo + hi)
        f, _ = frac(mid)
        if abs(f - overlap) < best_err:
            best_shift, best_err = mid, abs(f - overlap)
        if f > overlap:
            lo = mid
        else:
            hi = mid
        if best_err < 0.005:
            break
    cam2 = cam1 + best_shift * side
    _, noisy2 = _kinect_view(rng, prims, cam2, target + best_shift * side)
    ref = noisy1[rng.choice(len(noisy1), size=n_ref, replace=len(noisy1) < n_ref)]
    src0 = noisy2[rng.choice(len(noisy2), size=n_src, replace=len(noisy2) < n_src)]
    src, theta = _move_source(rng, src0)
    return Pair("kinect", src.astype(np.float32), ref.astype(np.float32), theta,
                {"seed": seed, "overlap_target": overlap, "overlap_err": best_err,
                 "shift": best_shift})


# ---------------------------------------------------------------------------
# LiDAR-shaped street
# ---------------------------------------------------------------------------

def _street_scene(rng, length=90.0):
    prims = [("plane", ())]
    for side in (-1.0, 1.0):
        x = -length
        while x < length:
            w = rng.uniform(8.0, 20.0)
            y0 = rng.uniform(8.0, 12.0)
            depth = rng.uniform(8.0, 15.0)
            h = rng.uniform(6.0, 25.0)
            ylo, yhi = (y0, y0 + depth) if side > 0 else (-y0 - depth, -y0)
            prims.append(("box", (np.array([x, ylo, 0.0]), np.array([x + w, yhi, h]))))
            x += w + rng.uniform(1.0, 4.0)
        x = -length
        while x < length:
            x += rng.uniform(8.0, 15.0)
            prims.append(("cylinder", (x, side * rng.uniform(5.0, 6.5), rng.uniform(0.1, 0.2),
                                       0.0, rng.uniform(4.0, 8.0))))
    return prims


def _ring_rays(yaw, az_offset_deg=0.0):
    elev = np.deg2rad(np.linspace(-24.8, 2.0, 64))
    az = np.deg2rad(np.arange(1800) * 0.2 + az_offset_deg) + yaw
    e, a = np.meshgrid(elev, az, indexing="ij")
    d = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)], axis=-1)
    return d.reshape(-1, 3)


def _ring_scan(rng, prims, pos, yaw, n_needed, max_range=80.0, sigma=0.02):
    pts = []
    offset = 0.0
    total = 0
    while total < n_needed:
        d = _ring_rays(yaw, offset)
        t = _cast(pos, d, prims)
        keep = t <= max_range
        tn = t[keep] + rng.normal(0.0, sigma, size=int(keep.sum()))
        p = pos + tn[:, None] * d[keep]
        pts.append(p)
        total += len(p)
        offset += 0.1
    return np.concatenate(pts)


def lidar_pair(seed: int, n_src: int = 20000, n_ref: int = 100000) -> Pair:
    """64-beam ring scanner (elevations evenly spaced in [-24.8, +2] deg,
    0.2 deg azimuth, range <= 80 m, range noise sigma 2 cm) at 1.8 m height in
    a street of box buildings and pole cylinders. Reference: ``n_ref`` hits of
    the first scan (an extra sweep at +0.1 deg azimuth is added when one sweep
    is short). Source: ``n_src`` hits of a scan taken 1-3 m away with yaw
    U(+-10 deg), in its own sensor frame; ``theta_true`` is that relative pose."""
    rng, _, _ = rng_streams(seed)
    prims = _street_scene(rng)
    pos1 = np.array([0.0, 0.0, 1.8])
    dist = rng.uniform(1.0, 3.0)
    phi = rng.uniform(0, 2 * np.pi)
    yaw2 = np.deg2rad(rng.uniform(-10.0, 10.0))
    pos2 = pos1 + np.array([dist * np.cos(phi), dist * np.sin(phi), 0.0])
    scan1 = _ring_scan(rng, prims, pos1, 0.0, n_ref) - pos1
    scan2_world = _ring_scan(rng, prims, pos2, yaw2, n_src)
    rot2 = Rotation.from_euler("Z", yaw2)
    scan2 = rot2.inv().apply(scan2_world - pos2)
    ref = scan1[rng.choice(len(scan1), size=n_ref, replace=False)]
    src = scan2[rng.choice(len(scan2), size=n_src, replace=False)]
    t = pos2 - pos1
    theta = np.array([t[0], t[1], t[2], 0.0, 0.0, yaw2])
    return Pair("lidar", src.astype(np.float32), ref.astype(np.float32), theta,
                {"seed": seed, "sensor_offset": dist})


def resample_pair(pair: Pair, rng, n_src: int, n_ref: int) -> Pair:
    """Draw ``n_src`` source and ``n_ref`` reference points from a pair
    (without replacement when enough points exist)."""
    s = pair.src[rng.choice(len(pair.src), size=n_src, replace=len(pair.src) < n_src)]
    r = pair.ref[rng.choice(len(pair.ref), size=n_ref, replace=len(pair.ref) < n_ref)]
    return Pair(pair.name, np.ascontiguousarray(s), np.ascontiguousarray(r),
                pair.theta_true.copy(), dict(pair.meta))


# ---------------------------------------------------------------------------
# random numbers the method draws: initial particles and minibatches
# ---------------------------------------------------------------------------

def init_particles(seed: int, K: int, half_trans: float = 0.2,
                   half_rot: float = np.pi / 4, centre=None) -> np.ndarray:
    """K x 6 float64 particles, uniform in centre +- (half_trans, half_rot)."""
    _, rng, _ = rng_streams(seed)
    c = np.zeros(6) if centre is None else np.asarray(centre, dtype=np.float64)
    half = np.array([half_trans] * 3 + [half_rot] * 3)
    return c[None, :] + rng.uniform(-1.0, 1.0, size=(K, 6)) * half[None, :]


def minibatch_schedule(seed: int, N: int, m: int, T: int) -> np.ndarray:
    """T x m int32: row t holds m distinct source indices drawn uniformly
    without replacement, fresh for each iteration."""
    if not (1 <= m <= N):
        raise ValueError("need 1 <= m <= N")
    _, _, rng = rng_streams(seed)
    out = np.empty((T, m), dtype=np.int32)
    for t in range(T):
        out[t] = rng.choice(N, size=m, replace=False)
    return out
