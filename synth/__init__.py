"""Seeded synthetic maps and LiDAR scans for the 3D-BBS localization workloads.

This module only produces inputs: point clouds of a map, scans taken from a known
pose, and the search ranges that go with them.  It holds none of the method's
arithmetic (no voxel keys, no scores, no search); both the HIP library and the
CPU oracle consume exactly the arrays produced here.

The paper evaluates on a simulated urban map (Sec. IV-A) and a real outdoor map
(Sec. IV-B), neither of which is available.  The generators below stand in for
them: an indoor box room with pillars, and a procedural city of building blocks,
streets, poles and ground, both scanned by an analytic ray caster with the
geometry of a multi-beam spinning LiDAR.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Scene", "Scan", "room_scene", "city_scene", "scan_scene", "rotation_zyx",
    "search_range_room", "search_range_city", "threshold_95", "tiny_scene", "city_query", "room_query",
]


@dataclasses.dataclass
class Scene:
    """A map: surface samples plus the analytic geometry used for ray casting."""
    points: np.ndarray          # (N, 3) float32 map points
    boxes: np.ndarray           # (B, 6) float64 [xmin, ymin, zmin, xmax, ymax, zmax]
    ground: tuple               # (xmin, ymin, xmax, ymax) of the z = 0 ground plane, or None
    walls_box: tuple | None     # inner room box (x0, y0, x1, y1, z1) whose walls face inward, or None
    extent: tuple               # (xmin, ymin, zmin, xmax, ymax, zmax) of the map
    streets: np.ndarray | None  # (S, 5) [x0, y0, x1, y1, half_width] street centre segments, or None
    seed: int = 0


@dataclasses.dataclass
class Scan:
    points: np.ndarray          # (K, 3) float32, sensor frame
    pose: np.ndarray            # (6,) float64 true pose x, y, z, roll, pitch, yaw
    seed: int = 0


def rotation_zyx(roll: float, pitch: float, yaw: float) -> np.ndarray:
    """Rotation Rz(yaw) @ Ry(pitch) @ Rx(roll) in float64 (sensor -> world)."""
    ca, sa = math.cos(roll), math.sin(roll)
    cb, sb = math.cos(pitch), math.sin(pitch)
    cg, sg = math.cos(yaw), math.sin(yaw)
    rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]], dtype=np.float64)
    ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]], dtype=np.float64)
    rz = np.array([[cg, -sg, 0], [sg, cg, 0], [0, 0, 1]], dtype=np.float64)
    return rz @ ry @ rx


def threshold_95(k: int) -> int:
    """Score threshold at 95 % of the scan points, rounded up, in integers."""
    return (95 * k + 99) // 100


# --------------------------------------------------------------------------- surfaces

def _grid(a0, a1, step):
    n = int(math.floor((a1 - a0) / step + 1e-9)) + 1
    return a0 + step * np.arange(n, dtype=np.float64)


def _sample_box_faces(box, step, with_top=True, with_bottom=False):
    """Lattice samples on the faces of an axis-aligned box."""
    x0, y0, z0, x1, y1, z1 = box
    xs, ys, zs = _grid(x0, x1, step), _grid(y0, y1, step), _grid(z0, z1, step)
    out = []
    # x faces
    Y, Z = np.meshgrid(ys, zs, indexing="ij")
    for x in (x0, x1):
        out.append(np.stack([np.full(Y.size, x), Y.ravel(), Z.ravel()], 1))
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    for y in (y0, y1):
        out.append(np.stack([X.ravel(), np.full(X.size, y), Z.ravel()], 1))
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    if with_top:
        out.append(np.stack([X.ravel(), Y.ravel(), np.full(X.size, z1)], 1))
    if with_bottom:
        out.append(np.stack([X.ravel(), Y.ravel(), np.full(X.size, z0)], 1))
    return np.concatenate(out, 0)


# --------------------------------------------------------------------------- room

def room_scene(seed: int = 0, size: float = 20.0, height: float = 5.0, n_pillars: int = 8,
               step: float = 0.1) -> Scene:
    """Box room [-size/2, size/2]^2 x [0, height]: floor, four walls, pillars.

    Surfaces are lattice-sampled every `step` metres.  Pillars are square boxes
    of seeded centre and a side drawn from U(0.3, 0.6) m, floor to ceiling height.
    """
    rng = np.random.default_rng(seed)
    h = size / 2
    pts = []
    xs = _grid(-h, h, step)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    pts.append(np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1))          # floor
    zs = _grid(0.0, height, step)
    A, Z = np.meshgrid(xs, zs, indexing="ij")
    for c in (-h, h):
        pts.append(np.stack([np.full(A.size, c), A.ravel(), Z.ravel()], 1))    # walls x = +-h
        pts.append(np.stack([A.ravel(), np.full(A.size, c), Z.ravel()], 1))    # walls y = +-h
    boxes = []
    for _ in range(n_pillars):
        w = rng.uniform(0.3, 0.6)
        cx, cy = rng.uniform(-h + 1.5, h - 1.5, size=2)
        b = (cx - w / 2, cy - w / 2, 0.0, cx + w / 2, cy + w / 2, height)
        boxes.append(b)
        pts.append(_sample_box_faces(b, step, with_top=False))
    points = np.concatenate(pts, 0).astype(np.float32)
    return Scene(points=points, boxes=np.array(boxes, dtype=np.float64).reshape(-1, 6),
                 ground=(-h, -h, h, h), walls_box=(-h, -h, h, h, height),
                 extent=(-h, -h, 0.0, h, h, height), streets=None, seed=seed)


def search_range_room(size: float = 20.0, z_centre: float = 1.5, z_half: float = 0.5,
                      rp_deg: float = 2.0):
    """Search ranges (min[6], max[6]) for the room: x, y over the room, z +-0.5 m
    around the nominal sensor height, roll/pitch +-2 deg, yaw [0, 2 pi)."""
    h = size / 2
    rp = math.radians(rp_deg)
    lo = np.array([-h, -h, z_centre - z_half, -rp, -rp, 0.0], dtype=np.float32)
    hi = np.array([h, h, z_centre + z_half, rp, rp, 2 * math.pi], dtype=np.float32)
    return lo, hi


# --------------------------------------------------------------------------- city

def city_scene(seed: int = 1000, half: float = 250.0, pitch: float = 50.0, street: float = 12.0,
               step: float = 0.25, hmin: float = 8.0, hmax: float = 30.0) -> Scene:
    """Procedural city on [-half, half]^2: ground, a block grid of buildings, poles.

    Streets of width `street` run along the lines x, y = -half + i * pitch.  Each
    block holds one to four box buildings of seeded footprint and height in
    [hmin, hmax]; poles (0.3 m square, 6-8 m tall) stand along the street sides.
    Surfaces (ground outside footprints, walls, roofs, poles) are lattice-sampled
    every `step` metres.
    """
    rng = np.random.default_rng(seed)
    nb = int(round(2 * half / pitch))
    boxes = []
    margin = street / 2 + 1.0
    for i in range(nb):
        for j in range(nb):
            bx0, by0 = -half + i * pitch + margin, -half + j * pitch + margin
            bx1, by1 = -half + (i + 1) * pitch - margin, -half + (j + 1) * pitch - margin
            split = rng.integers(0, 4)   # 0: one building, 1: split x, 2: split y, 3: both
            xs = [bx0, bx1] if split in (0, 2) else [bx0, (bx0 + bx1) / 2 - 1.5, (bx0 + bx1) / 2 + 1.5, bx1]
            ys = [by0, by1] if split in (0, 1) else [by0, (by0 + by1) / 2 - 1.5, (by0 + by1) / 2 + 1.5, by1]
            for a in range(0, len(xs), 2):
                for b in range(0, len(ys), 2):
                    lx0, lx1, ly0, ly1 = xs[a], xs[a + 1], ys[b], ys[b + 1]
                    # shrink the lot by a seeded setback on each side
                    s = rng.uniform(0.0, 3.0, size=4)
                    x0, x1 = lx0 + s[0], lx1 - s[1]
                    y0, y1 = ly0 + s[2], ly1 - s[3]
                    if x1 - x0 < 4 or y1 - y0 < 4:
                        continue
                    hgt = rng.uniform(hmin, hmax)
                    boxes.append((_snap(x0, step), _snap(y0, step), 0.0,
                                  _snap(x1, step), _snap(y1, step), _snap(hgt, step)))
    buildings = np.array(boxes, dtype=np.float64)
    poles = []
    for k in range(nb + 1):
        line = -half + k * pitch
        for side in (-1, 1):
            off = line + side * (street / 2 - 0.5)
            if abs(off) > half - 1:
                continue
            along = -half + 10.0
            while along < half - 10.0:
                along += rng.uniform(18.0, 32.0)
                if along > half - 10.0:
                    break
                hp = _snap(rng.uniform(6.0, 8.0), step)
                for (px, py) in ((off, along), (along, off)):
                    poles.append((_snap(px - 0.15, step / 5), _snap(py - 0.15, step / 5), 0.0,
                                  _snap(px + 0.15, step / 5), _snap(py + 0.15, step / 5), hp))
    poles = np.array(poles, dtype=np.float64).reshape(-1, 6)
    all_boxes = np.concatenate([buildings, poles], 0)

    pts = []
    g = _grid(-half, half, step)
    X, Y = np.meshgrid(g, g, indexing="ij")
    X, Y = X.ravel(), Y.ravel()
    inside = np.zeros(X.size, dtype=bool)
    for b in buildings:
        inside |= (X > b[0]) & (X < b[3]) & (Y > b[1]) & (Y < b[4])
    pts.append(np.stack([X[~inside], Y[~inside], np.zeros((~inside).sum())], 1))
    for b in buildings:
        pts.append(_sample_box_faces(b, step, with_top=True))
    for b in poles:
        pts.append(_sample_box_faces(b, 0.1, with_top=True))
    points = np.concatenate(pts, 0).astype(np.float32)
    streets = []
    for k in range(nb + 1):
        line = -half + k * pitch
        streets.append((line, -half, line, half, street / 2))
        streets.append((-half, line, half, line, street / 2))
    return Scene(points=points, boxes=all_boxes, ground=(-half, -half, half, half), walls_box=None,
                 extent=(-half, -half, 0.0, half, half, float(all_boxes[:, 5].max())),
                 streets=np.array(streets, dtype=np.float64), seed=seed)


def _snap(v, step):
    return round(v / step) * step


def search_range_city(half: float = 250.0, z_centre: float = 1.8, z_half: float = 2.0,
                      rp_deg: float = 3.0):
    """Search ranges for the city: +-half in x, y, +-z_half around the nominal
    sensor height, roll/pitch +-rp_deg, yaw [0, 2 pi)."""
    rp = math.radians(rp_deg)
    lo = np.array([-half, -half, z_centre - z_half, -rp, -rp, 0.0], dtype=np.float32)
    hi = np.array([half, half, z_centre + z_half, rp, rp, 2 * math.pi], dtype=np.float32)
    return lo, hi


# --------------------------------------------------------------------------- ray casting

def _ray_cast(scene: Scene, origin: np.ndarray, dirs: np.ndarray, max_range: float) -> np.ndarray:
    """Nearest hit distance of each ray (inf where nothing is hit within range)."""
    n = dirs.shape[0]
    best = np.full(n, np.inf)
    d = dirs
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
    # ground plane z = 0 inside the ground rectangle
    if scene.ground is not None:
        t = np.where(d[:, 2] < 0, -origin[2] / d[:, 2], np.inf)
        hx, hy = origin[0] + t * d[:, 0], origin[1] + t * d[:, 1]
        gx0, gy0, gx1, gy1 = scene.ground
        ok = (t > 1e-6) & (hx >= gx0) & (hx <= gx1) & (hy >= gy0) & (hy <= gy1)
        best = np.where(ok, np.minimum(best, t), best)
    # inward-facing room walls
    if scene.walls_box is not None:
        x0, y0, x1, y1, z1 = scene.walls_box
        for axis, lo, hi in ((0, x0, x1), (1, y0, y1)):
            for plane in (lo, hi):
                t = (plane - origin[axis]) * inv[:, axis]
                p = origin[None, :] + t[:, None] * d
                o = 1 - axis
                ok = (t > 1e-6) & (p[:, 2] >= 0) & (p[:, 2] <= z1) & (p[:, o] >= [x0, y0][o]) & \
                     (p[:, o] <= [x1, y1][o])
                best = np.where(ok, np.minimum(best, t), best)
    # boxes (slab test), only those that can be reached; rays are bucketed by
    # azimuth sector and tested against the boxes whose angular extent (seen
    # from the origin, with a margin) overlaps the sector.  A ray can only hit
    # a box whose footprint its horizontal direction crosses, so the culling
    # changes no hit.
    if len(scene.boxes):
        b = scene.boxes
        cx = np.clip(origin[0], b[:, 0], b[:, 3])
        cy = np.clip(origin[1], b[:, 1], b[:, 4])
        near = np.hypot(cx - origin[0], cy - origin[1]) <= max_range
        b = b[near]
        n_sec = 256
        phi = np.arctan2(d[:, 1], d[:, 0])
        sec = np.floor((phi + np.pi) / (2 * np.pi) * n_sec).astype(np.int64) % n_sec
        corners = np.stack([np.stack([b[:, 0], b[:, 1]], 1), np.stack([b[:, 3], b[:, 1]], 1),
                            np.stack([b[:, 0], b[:, 4]], 1), np.stack([b[:, 3], b[:, 4]], 1)], 1)
        rel = corners - origin[None, None, :2]
        mid = rel.mean(axis=1)
        phc = np.arctan2(mid[:, 1], mid[:, 0])
        ang = np.arctan2(rel[:, :, 1], rel[:, :, 0]) - phc[:, None]
        ang = (ang + np.pi) % (2 * np.pi) - np.pi
        inside = (origin[0] >= b[:, 0]) & (origin[0] <= b[:, 3]) & (origin[1] >= b[:, 1]) & (origin[1] <= b[:, 4])
        half = np.where(inside, np.pi, np.abs(ang).max(axis=1)) + 4 * np.pi / n_sec
        order = np.argsort(sec, kind="stable")
        bounds = np.searchsorted(sec[order], np.arange(n_sec + 1))
        for k in range(n_sec):
            rays = order[bounds[k]:bounds[k + 1]]
            if len(rays) == 0:
                continue
            psi = -np.pi + (k + 0.5) * 2 * np.pi / n_sec
            dd = np.abs((psi - phc + np.pi) % (2 * np.pi) - np.pi)
            cand = b[dd <= half]
            if len(cand) == 0:
                continue
            chunk = max(1, int(2e7 // len(cand)))
            for s0 in range(0, len(rays), chunk):
                rr = rays[s0:s0 + chunk]
                iv = inv[rr]
                t1 = (cand[None, :, 0:3] - origin[None, None, :]) * iv[:, None, :]
                t2 = (cand[None, :, 3:6] - origin[None, None, :]) * iv[:, None, :]
                tmin = np.nanmax(np.minimum(t1, t2), axis=2)
                tmax = np.nanmin(np.maximum(t1, t2), axis=2)
                hit = (tmax >= tmin) & (tmax > 1e-6)
                tt = np.where(hit, np.where(tmin > 1e-6, tmin, np.inf), np.inf)
                best[rr] = np.minimum(best[rr], tt.min(axis=1))
    best[best > max_range] = np.inf
    return best


def _lidar_dirs(n_beams, n_az, elev_lo_deg, elev_hi_deg):
    el = np.radians(np.linspace(elev_lo_deg, elev_hi_deg, n_beams))
    az = np.linspace(0.0, 2 * np.pi, n_az, endpoint=False)
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1).reshape(-1, 3)


def _free_position(scene: Scene, rng, z: float, clearance: float = 0.5):
    """A random sensor position that is not inside or next to any box."""
    x0, y0, _, x1, y1, _ = scene.extent
    for _ in range(10000):
        if scene.streets is not None:
            s = scene.streets[rng.integers(len(scene.streets))]
            t = rng.uniform(0.1, 0.9)
            px, py = s[0] + t * (s[2] - s[0]), s[1] + t * (s[3] - s[1])
            off = rng.uniform(-s[4] + 2.0, s[4] - 2.0)
            if s[0] == s[2]:
                px += off
            else:
                py += off
        else:
            px = rng.uniform(x0 + 2.0, x1 - 2.0)
            py = rng.uniform(y0 + 2.0, y1 - 2.0)
        b = scene.boxes
        inside = (px > b[:, 0] - clearance) & (px < b[:, 3] + clearance) & \
                 (py > b[:, 1] - clearance) & (py < b[:, 4] + clearance) if len(b) else np.zeros(0, bool)
        if not inside.any() and x0 + 1 < px < x1 - 1 and y0 + 1 < py < y1 - 1:
            return px, py, z
    raise RuntimeError("no free sensor position found")


def scan_scene(scene: Scene, seed: int, n_points: int, *, z: float, z_jitter: float = 0.0,
               rp_deg: float = 2.0, noise: float = 0.02, n_beams: int = 32, n_az: int = 1024,
               elev=(-25.0, 15.0), max_range: float = 100.0, voxel: float = 0.0,
               pose: np.ndarray | None = None) -> Scan:
    """Ray-cast a spinning-LiDAR scan of `scene` from a seeded random pose.

    The pose is x, y on free ground (streets for a city), z = `z` + U(-z_jitter,
    z_jitter), roll and pitch U(-rp_deg, rp_deg) degrees, yaw U[0, 2 pi).  Hits
    are expressed in the sensor frame, optionally thinned by a voxel grid of
    `voxel` metres, trimmed at random to exactly `n_points` and perturbed by iid
    N(0, noise^2) per coordinate.
    """
    rng = np.random.default_rng(seed)
    if pose is None:
        px, py, pz = _free_position(scene, rng, z + rng.uniform(-z_jitter, z_jitter) if z_jitter else z)
        rp = math.radians(rp_deg)
        roll, pitch = rng.uniform(-rp, rp, size=2)
        yaw = rng.uniform(0.0, 2 * math.pi)
        pose = np.array([px, py, pz, roll, pitch, yaw], dtype=np.float64)
    R = rotation_zyx(pose[3], pose[4], pose[5])
    dirs_s = _lidar_dirs(n_beams, n_az, *elev)
    dirs_w = dirs_s @ R.T
    t = _ray_cast(scene, pose[:3], dirs_w, max_range)
    ok = np.isfinite(t)
    pts_s = dirs_s[ok] * t[ok, None]
    if voxel > 0:
        keys = np.floor(pts_s / voxel).astype(np.int64)
        _, first = np.unique(keys, axis=0, return_index=True)
        pts_s = pts_s[np.sort(first)]
    if len(pts_s) == 0:
        raise RuntimeError("scan hit nothing")
    replace = len(pts_s) < n_points
    idx = rng.choice(len(pts_s), size=n_points, replace=replace)
    pts = pts_s[idx] + (rng.normal(0.0, noise, size=(n_points, 3)) if noise > 0 else 0.0)
    return Scan(points=pts.astype(np.float32), pose=pose, seed=seed)


def city_query(scene: Scene, seed: int, n_points: int, voxel: float = 0.5) -> Scan:
    """A query scan of the city workload: 64 beams over -25..+15 deg, 2048
    azimuths, 100 m range, from a street position at 1.8 m with roll and pitch
    U(-3, 3) deg and uniform yaw, voxel-thinned at `voxel` metres, trimmed to
    `n_points`, N(0, 0.02 m) noise."""
    return scan_scene(scene, seed, n_points, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048, voxel=voxel)


def room_query(scene: Scene, seed: int, n_points: int = 2000) -> Scan:
    """A query scan of the indoor workload: 32 beams x 1024 azimuths from
    z = 1.5 +- 0.25 m with roll and pitch U(-2, 2) deg and uniform yaw."""
    return scan_scene(scene, seed, n_points, z=1.5, z_jitter=0.25, rp_deg=2.0)


# --------------------------------------------------------------------------- tiny

def tiny_scene(seed: int = 0, n_map: int = 600, extent: float = 6.0) -> Scene:
    """A small random scene for exhaustive tests: a floor patch plus a few boxes,
    sampled at 0.25 m, inside [-extent, extent]^2 x [0, 3]."""
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(4):
        w, d = rng.uniform(0.5, 2.0, size=2)
        cx, cy = rng.uniform(-extent + 1.5, extent - 1.5, size=2)
        boxes.append((_snap(cx - w / 2, 0.25), _snap(cy - d / 2, 0.25), 0.0,
                      _snap(cx + w / 2, 0.25), _snap(cy + d / 2, 0.25), _snap(rng.uniform(1.0, 3.0), 0.25)))
    pts = [np.array(_sample_box_faces(b, 0.25)) for b in boxes]
    g = _grid(-extent, extent, 0.5)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts.append(np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1))
    points = np.concatenate(pts, 0)
    if n_map and len(points) > n_map:
        points = points[rng.choice(len(points), size=n_map, replace=False)]
    return Scene(points=points.astype(np.float32), boxes=np.array(boxes), ground=(-extent, -extent, extent, extent),
                 walls_box=None, extent=(-extent, -extent, 0.0, extent, extent, 3.0), streets=None, seed=seed)
