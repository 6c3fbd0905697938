"""Seeded synthetic workloads: race-track LiDAR scans and voxelised maps.

This module only *generates inputs*.  It holds none of the neighbour-search or
covariance arithmetic, so both the GPU path and the CPU oracle can take their
inputs from here without sharing any of the method's code.

The paper's recordings (Ouster OS2-128 + 2x VLP-16 on one car, three Luminar
units on the other; Sec. IV-B platform tables) are not available, so every
workload is a stand-in with the same structure: a 128-ring spinning LiDAR
ray-cast against a stadium-shaped track (ground plane plus two 1 m walls 8 m
either side of the centreline), several sensors per frame, and a pre-built map
voxel-filtered the way Sec. III-D and the benchmark footnote of Sec. IV-E.3
describe ("voxel-filtered points", a leaf size).

All randomness is ``numpy.random.default_rng(seed)`` (PCG64).  Every array is
float32 ``[n, 3]`` C-contiguous.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Optional, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Track geometry: stadium (two 250 m straights, two r = 75 m semicircles),
# bounding box 400 m x 150 m, centreline perimeter 500 + 150*pi m.
# --------------------------------------------------------------------------
STRAIGHT = 250.0
BEND_R = 75.0
WALL_OFFSET = 8.0
WALL_HEIGHT = 1.0
SENSOR_HEIGHT = 1.2
PERIMETER = 2.0 * STRAIGHT + 2.0 * math.pi * BEND_R

# spinning LiDAR: 128 rings over [-22.5, -0.6] deg elevation, 1024 azimuths
N_RINGS = 128
N_AZIMUTHS = 1024
ELEV_MIN_DEG = -22.5
ELEV_MAX_DEG = -0.6
RANGE_MIN = 0.5
RANGE_MAX = 120.0
RANGE_SIGMA = 0.02


def centreline_pose(s: np.ndarray | float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Arc length ``s`` (m, any real) -> centreline (x, y, yaw), counter-clockwise."""
    s = np.mod(np.asarray(s, dtype=np.float64), PERIMETER)
    x = np.empty_like(s)
    y = np.empty_like(s)
    yaw = np.empty_like(s)
    arc = math.pi * BEND_R
    s1, s2, s3 = STRAIGHT, STRAIGHT + arc, 2 * STRAIGHT + arc
    m = s < s1                                   # bottom straight, heading +x
    x[m], y[m], yaw[m] = -STRAIGHT / 2 + s[m], -BEND_R, 0.0
    m = (s >= s1) & (s < s2)                     # right bend, centre (+125, 0)
    phi = (s[m] - s1) / BEND_R
    x[m] = STRAIGHT / 2 + BEND_R * np.cos(phi - math.pi / 2)
    y[m] = BEND_R * np.sin(phi - math.pi / 2)
    yaw[m] = phi
    m = (s >= s2) & (s < s3)                     # top straight, heading -x
    x[m], y[m], yaw[m] = STRAIGHT / 2 - (s[m] - s2), BEND_R, math.pi
    m = s >= s3                                  # left bend, centre (-125, 0)
    phi = (s[m] - s3) / BEND_R
    x[m] = -STRAIGHT / 2 + BEND_R * np.cos(phi + math.pi / 2)
    y[m] = BEND_R * np.sin(phi + math.pi / 2)
    yaw[m] = phi + math.pi
    return x, y, yaw


def track_pose(s: float, lateral: float = 0.0, yaw_noise: float = 0.0):
    """Pose on the track: centreline point shifted ``lateral`` m to the left."""
    x, y, yaw = centreline_pose(s)
    x, y, yaw = float(x), float(y), float(yaw)
    x -= lateral * math.sin(yaw)
    y += lateral * math.cos(yaw)
    return x, y, yaw + yaw_noise


def _wall_hits(ox, oy, ux, uy):
    """Horizontal distance along the ray to every wall piece (inf if missed)."""
    half = STRAIGHT / 2
    best = np.full(ox.shape, np.inf)
    for radius in (BEND_R - WALL_OFFSET, BEND_R + WALL_OFFSET):
        for side in (-1.0, 1.0):                 # straights y = +-radius
            with np.errstate(divide="ignore", invalid="ignore"):
                s = (side * radius - oy) / uy
            xh = ox + s * ux
            ok = (s > 1e-9) & (np.abs(xh) <= half)
            best = np.where(ok & (s < best), s, best)
        for cx in (-half, half):                 # semicircles
            wx, wy = ox - cx, oy
            b = ux * wx + uy * wy
            c = wx * wx + wy * wy - radius * radius
            disc = b * b - c
            root = np.sqrt(np.maximum(disc, 0.0))
            for s in (-b - root, -b + root):
                xh = ox + s * ux
                on_arc = (xh >= half) if cx > 0 else (xh <= -half)
                ok = (disc >= 0) & (s > 1e-9) & on_arc
                best = np.where(ok & (s < best), s, best)
    return best


@dataclasses.dataclass
class Scan:
    points_sensor: np.ndarray   # float32 [n, 3], sensor frame
    points_world: np.ndarray    # float32 [n, 3], world frame
    pose: Tuple[float, float, float]


_ELEV = np.deg2rad(np.linspace(ELEV_MIN_DEG, ELEV_MAX_DEG, N_RINGS))
_AZIM = 2.0 * math.pi * np.arange(N_AZIMUTHS) / N_AZIMUTHS


def raycast_scan(pose, rng: np.random.Generator, dropout: float = 0.1,
                 yaw_offset: float = 0.0) -> Scan:
    """One 128 x 1024 spinning-LiDAR sweep from ``pose`` = (x, y, yaw).

    Rays are emitted azimuth-major (for each azimuth, all rings), as a
    spinning unit streams its columns.  Each ray returns its nearest hit among
    the ground plane z = 0 and the two walls, with N(0, 2 cm) range noise;
    rays are dropped i.i.d. with probability ``dropout`` and returns outside
    [0.5, 120] m are discarded.  ``yaw_offset`` is the sensor's mounting yaw
    on the vehicle; ``points_sensor`` is in the vehicle frame (sensor at the
    origin, ground at z = -1.2 m).
    """
    px, py, yaw = pose
    th = _AZIM + yaw + yaw_offset                      # world heading per azimuth
    ux, uy = np.cos(th), np.sin(th)
    s_wall = _wall_hits(np.full(th.shape, px), np.full(th.shape, py), ux, uy)
    ce, se = np.cos(_ELEV), np.sin(_ELEV)
    t_ground = SENSOR_HEIGHT / (-se)                    # [rings]
    t_wall = s_wall[:, None] / ce[None, :]              # [azimuths, rings]
    z_wall = SENSOR_HEIGHT + t_wall * se[None, :]
    wall_ok = np.isfinite(t_wall) & (z_wall >= 0.0) & (z_wall <= WALL_HEIGHT)
    t_hit = np.where(wall_ok & (t_wall < t_ground[None, :]), t_wall, t_ground[None, :]).ravel()
    r = t_hit + rng.normal(0.0, RANGE_SIGMA, size=t_hit.shape)
    keep = (rng.random(size=t_hit.shape) >= dropout) & (r >= RANGE_MIN) & (r <= RANGE_MAX)
    ai, ei = np.nonzero(keep.reshape(N_AZIMUTHS, N_RINGS))
    rk = r[keep]
    a_v = _AZIM[ai] + yaw_offset
    pv = np.empty((rk.size, 3))
    pv[:, 0] = rk * ce[ei] * np.cos(a_v)
    pv[:, 1] = rk * ce[ei] * np.sin(a_v)
    pv[:, 2] = rk * se[ei]
    c, s = math.cos(yaw), math.sin(yaw)
    pw = np.empty_like(pv)
    pw[:, 0] = px + c * pv[:, 0] - s * pv[:, 1]
    pw[:, 1] = py + s * pv[:, 0] + c * pv[:, 1]
    pw[:, 2] = SENSOR_HEIGHT + pv[:, 2]
    return Scan(np.ascontiguousarray(pv, np.float32),
                np.ascontiguousarray(pw, np.float32), (px, py, yaw + yaw_offset))


# --------------------------------------------------------------------------
# Config 1: plane + wall
# --------------------------------------------------------------------------
def plane_wall(n: int = 2048, seed: int = 0) -> np.ndarray:
    """70 % of points on z = 0 over [-10,10]^2, 30 % on the wall x = 5 m."""
    rng = np.random.default_rng(seed)
    n_plane = int(math.floor(0.7 * n))
    n_wall = n - n_plane
    plane = np.stack([rng.uniform(-10, 10, n_plane), rng.uniform(-10, 10, n_plane),
                      rng.normal(0, 0.02, n_plane)], axis=1)
    wall = np.stack([5.0 + rng.normal(0, 0.02, n_wall), rng.uniform(-10, 10, n_wall),
                     rng.uniform(0, 2, n_wall)], axis=1)
    return np.ascontiguousarray(np.concatenate([plane, wall]), np.float32)


# --------------------------------------------------------------------------
# Config 2: one scan, sensor frame
# --------------------------------------------------------------------------
def single_scan(seed: int = 1, dropout: float = 0.1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.0, PERIMETER)
    pose = track_pose(s)
    return raycast_scan(pose, rng, dropout=dropout).points_sensor


# --------------------------------------------------------------------------
# Config 3: voxelised map + source scan
# --------------------------------------------------------------------------
VOXEL = 0.2
VOXEL_ORIGIN = np.array([0.0, 0.0, -0.1])


# dense voxel index over a fixed world box that contains every return from a
# track pose (|x| <= 200 + 120 m, |y| <= 83 + 120 m, z in [-0.1, 1.1] m)
_VBOX_LO = np.array([-400.0, -250.0, -0.1 - 2 * VOXEL])
_VBOX_N = np.array([4000, 2500, 16], np.int64)


def _voxel_dense_index(p: np.ndarray) -> np.ndarray:
    v = np.floor((p.astype(np.float64) - _VBOX_LO) / VOXEL).astype(np.int64)
    if (v < 0).any() or (v >= _VBOX_N).any():
        raise ValueError("point outside the voxel box")
    return (v[:, 0] * _VBOX_N[1] + v[:, 1]) * _VBOX_N[2] + v[:, 2]


def _cache_dir() -> Optional[str]:
    d = os.environ.get("LKC_WORKLOAD_CACHE", "/tmp/lkc_workload_cache")
    try:
        os.makedirs(d, exist_ok=True)
        return d
    except OSError:
        return None


def _scan_world(args):
    seed, i, s, lateral = args
    rng = np.random.default_rng([seed, i])
    return raycast_scan(track_pose(s, lateral), rng).points_world


def build_map(n_points: int = 2_000_000, seed: int = 2, n_even: int = 40,
              use_cache: bool = True) -> Tuple[np.ndarray, int]:
    """Voxelised track map with exactly ``n_points`` voxel centroids.

    ``n_even`` scans at evenly spaced centreline poses are accumulated in the
    world frame; seeded random track poses (lateral offset U[-6, 6] m) are
    added in batches of 16 until at least ``n_points`` voxels (0.2 m, origin
    (0, 0, -0.1)) are occupied.  Each occupied voxel contributes the centroid
    of its returns; a seeded uniform subset of exactly ``n_points`` centroids
    is kept, in first-occupied order.  Scan i draws from
    ``default_rng([seed, i])``.  Returns (points float32 [n_points, 3],
    number of scans used).
    """
    from concurrent.futures import ThreadPoolExecutor
    cache = _cache_dir() if use_cache else None
    path = None
    if cache:
        path = os.path.join(cache, f"map_n{n_points}_s{seed}_e{n_even}_v3.npz")
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                return z["points"], int(z["n_scans"])
    rng = np.random.default_rng(seed)
    lut = np.full(int(np.prod(_VBOX_N)), -1, np.int32)
    cap = max(n_points * 2, 1 << 20)
    sums = np.zeros((cap, 3))
    cnts = np.zeros(cap)
    n_vox = 0
    n_scans = 0
    jobs = [(seed, i, i * PERIMETER / n_even, 0.0) for i in range(n_even)]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        while True:
            batch = list(ex.map(_scan_world, jobs))
            n_scans += len(batch)
            for pw in (np.concatenate(batch),):
                d = _voxel_dense_index(pw)
                slot = lut[d]
                new = slot < 0
                if new.any():
                    nd = np.unique(d[new])
                    if n_vox + nd.size > cap:
                        grow = max(cap, nd.size)
                        sums = np.concatenate([sums, np.zeros((grow, 3))])
                        cnts = np.concatenate([cnts, np.zeros(grow)])
                        cap += grow
                    lut[nd] = np.arange(n_vox, n_vox + nd.size, dtype=np.int32)
                    n_vox += nd.size
                    slot = lut[d]
                cnts[:n_vox] += np.bincount(slot, minlength=n_vox)
                for a in range(3):
                    sums[:n_vox, a] += np.bincount(slot, weights=pw[:, a], minlength=n_vox)
            if n_vox >= n_points:
                break
            jobs = [(seed, n_scans + j, rng.uniform(0, PERIMETER), rng.uniform(-6.0, 6.0))
                    for j in range(16)]
    cen = sums[:n_vox] / cnts[:n_vox, None]
    pick = np.sort(rng.choice(n_vox, size=n_points, replace=False))
    out = np.ascontiguousarray(cen[pick], np.float32)
    if path:
        tmp = path + f".tmp{os.getpid()}"
        np.savez(tmp, points=out, n_scans=np.int64(n_scans))
        os.replace(tmp + ".npz", path)
    return out, n_scans


def source_scan(n: int = 65_536, seed: int = 3, dropout: float = 0.1) -> np.ndarray:
    """A scan at a random track pose, ``n`` points kept in scan order, world frame."""
    rng = np.random.default_rng(seed)
    pose = track_pose(rng.uniform(0, PERIMETER), rng.uniform(-6.0, 6.0),
                      math.radians(rng.normal(0.0, 2.0)))
    sc = raycast_scan(pose, rng, dropout=dropout)
    keep = np.sort(rng.choice(sc.points_world.shape[0], size=n, replace=False))
    return np.ascontiguousarray(sc.points_world[keep])


# --------------------------------------------------------------------------
# Config 4: 16 frames x 3 sensors of uneven size
# --------------------------------------------------------------------------
def batched_scans(n_frames: int = 16, seed: int = 4, n_min: int = 20_000,
                  n_max: int = 131_072, spacing: float = 2.0) -> List[np.ndarray]:
    """Three sensors per frame (yaw offsets 0, +-120 deg), frames 2 m apart.

    Each scan is a seeded subset (scan order kept) of a 0 %-dropout sweep, of
    size drawn uniformly from {n_min..n_max}; points in the world frame.
    """
    rng = np.random.default_rng(seed)
    s0 = rng.uniform(0, PERIMETER)
    out = []
    for f in range(n_frames):
        pose = track_pose(s0 + f * spacing)
        for off in (0.0, 2 * math.pi / 3, -2 * math.pi / 3):
            sc = raycast_scan(pose, rng, dropout=0.0, yaw_offset=off)
            n = int(rng.integers(n_min, n_max + 1))
            n = min(n, sc.points_world.shape[0])
            keep = np.sort(rng.choice(sc.points_world.shape[0], size=n, replace=False))
            out.append(np.ascontiguousarray(sc.points_world[keep]))
    return out


# --------------------------------------------------------------------------
# Config 5: served stream
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    t_arrival: float     # seconds from stream start
    sensor: int
    map_id: int
    n_points: int
    scan_seed: int


SERVED_MAP_SIZES = (500_000, 1_000_000, 2_000_000, 4_000_000)


def served_schedule(duration: float = 60.0, rate_hz: float = 20.0, n_sensors: int = 3,
                    seed: int = 5, n_min: int = 10_000, n_max: int = 131_072,
                    n_maps: int = 4) -> List[Request]:
    """Poisson arrivals per sensor (exponential gaps, mean 1/rate), merged in time."""
    rng = np.random.default_rng(seed)
    reqs: List[Request] = []
    for sensor in range(n_sensors):
        t = 0.0
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= duration:
                break
            reqs.append(Request(t, sensor, int(rng.integers(0, n_maps)),
                                int(rng.integers(n_min, n_max + 1)),
                                int(rng.integers(0, 2**31 - 1))))
    reqs.sort(key=lambda r: (r.t_arrival, r.sensor))
    return reqs


def served_maps(sizes=SERVED_MAP_SIZES, seed: int = 50) -> List[np.ndarray]:
    """The resident maps of the served stream: same builder, different
    seeds; a size above 2,000,000 points is the union of two maps built
    with different seeds (a denser map of the same track)."""
    out = []
    for i, n in enumerate(sizes):
        parts, left, j = [], n, 0
        while left > 0:
            m = min(left, 2_000_000)
            parts.append(build_map(m, seed=seed + 10 * i + j)[0])
            left -= m
            j += 1
        out.append(np.ascontiguousarray(np.concatenate(parts)))
    return out


def served_scan_pool(n_poses: int = 16, seed: int = 6) -> List[np.ndarray]:
    """Full 0 %-dropout sweeps (131,072 points, world frame) of three
    sensors at n_poses random track poses; served requests take the first
    n points of pool[rid % len(pool)]."""
    rng = np.random.default_rng(seed)
    pool = []
    for _ in range(n_poses):
        pose = track_pose(rng.uniform(0, PERIMETER), rng.uniform(-6.0, 6.0))
        for off in (0.0, 2 * math.pi / 3, -2 * math.pi / 3):
            pool.append(raycast_scan(pose, rng, dropout=0.0, yaw_offset=off).points_world)
    return pool


def request_points(req: Request, map_seed_base: int = 100) -> np.ndarray:
    """World-frame points for a served request (scan at a random track pose)."""
    rng = np.random.default_rng(req.scan_seed)
    pose = track_pose(rng.uniform(0, PERIMETER), rng.uniform(-6.0, 6.0))
    sc = raycast_scan(pose, rng, dropout=0.0,
                      yaw_offset=2 * math.pi / 3 * req.sensor)
    n = min(req.n_points, sc.points_world.shape[0])
    keep = np.sort(rng.choice(sc.points_world.shape[0], size=n, replace=False))
    return np.ascontiguousarray(sc.points_world[keep])


# --------------------------------------------------------------------------
# Small structured clouds used by tests
# --------------------------------------------------------------------------
def lattice_1d(n: int = 64, a: float = 1.0) -> np.ndarray:
    p = np.zeros((n, 3), np.float32)
    p[:, 0] = a * np.arange(n, dtype=np.float32)
    return p


def lattice_nd(shape=(8, 8), a: float = 1.0) -> np.ndarray:
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    p = np.zeros((int(np.prod(shape)), 3), np.float32)
    for ax, g in enumerate(grids):
        p[:, ax] = a * g.ravel()
    return p


def random_cloud(n: int, seed: int, scale: float = 1.0, offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-scale, scale, (n, 3)) + np.asarray(offset),
                                np.float32)
