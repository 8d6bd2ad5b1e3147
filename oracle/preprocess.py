"""CPU oracle of the scan preprocessing that precedes the search.

TEST INFRASTRUCTURE ONLY (see `oracle/__init__.py`): only the tests, the
smoke check and the benchmark's CPU leg use it.

The paper names two steps before the search and leaves their arithmetic open:
- every scan is downsampled with a voxel-grid filter to about 1,000 points
  (Sec. IV, parameters);
- the scan is roughly aligned with gravity, in the real experiment along the
  average acceleration that the sensor's IMU measured (Sec. III-A; Sec. IV-B).

Readings (the library implements the same ones independently):
- Gravity alignment.  a = g / |g| (the measured acceleration, which points up
  when the sensor rests).  R is the smallest rotation taking a to +z:
      k = 1 / (1 + a_z)
      R = [[1 - k a_x a_x,  -k a_x a_y,    -a_x],
           [-k a_x a_y,     1 - k a_y a_y, -a_y],
           [a_x,            a_y,           a_z ]]
  (from R = I + [v]x + [v]x^2 / (1 + c) with v = a x z, c = a . z), every entry
  formed in double exactly as written and rounded once to float; a half turn
  about x, diag(1, -1, -1), when 1 + a_z < 1e-9.  Each output coordinate is
  (R_i0 x + R_i1 y) + R_i2 z in float32 with no contraction.
- Voxel-grid filter.  A point's voxel is floor(float32(p / leaf)) per axis.
  Every occupied voxel becomes the mean of its points.  Coordinates enter the
  sums as integers in units of 2^-24 m (round half to even of p * 2^24; the
  filter requires |p| < 1024 m), so the sums are exact and independent of
  their order; the mean is double(sum) / count * 2^-24, rounded once to float.
  Voxels come out in the order of their first point.  The leaf is at least
  2^-10 m, so voxel indices stay within +-2^20.
- Target size.  With target_points > 0 the leaf is chosen by 24 bisection
  steps in float: lo = 2^-10 m, hi = max(2 * extent, 1 m) where extent is the
  largest of the per-axis (max - min); mid = (lo + hi) * 0.5; a voxel count
  above the target moves lo to mid, otherwise hi; the leaf used is the final hi.
"""
from __future__ import annotations

import numpy as np

FIX_SCALE = float(2 ** 24)      # sum units: 2^-24 m
COORD_LIMIT = 1024.0            # |p| < 1024 m
BISECT_STEPS = 24
MIN_LEAF = 2.0 ** -10           # with |p| < 1024 m, voxel indices stay within +-2^20


def gravity_rotation(g) -> np.ndarray:
    """The float32 rotation of the gravity reading: a = g / |g| goes to +z."""
    gx, gy, gz = (float(v) for v in np.asarray(g, np.float32))
    norm = np.sqrt((gx * gx + gy * gy) + gz * gz)
    if not norm > 0.0:
        raise ValueError("gravity vector must be nonzero")
    ax, ay, az = gx / norm, gy / norm, gz / norm
    if 1.0 + az < 1e-9:
        R = np.diag([1.0, -1.0, -1.0])
    else:
        k = 1.0 / (1.0 + az)
        R = np.array([[1.0 - k * (ax * ax), -(k * (ax * ay)), -ax],
                      [-(k * (ax * ay)), 1.0 - k * (ay * ay), -ay],
                      [ax, ay, az]])
    return R.astype(np.float32)


def gravity_align(points, g) -> np.ndarray:
    """Rotate an n x 3 float32 scan by gravity_rotation(g)."""
    p = np.asarray(points, np.float32).reshape(-1, 3)
    R = gravity_rotation(g)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    out = np.empty_like(p)
    for i in range(3):
        out[:, i] = (R[i, 0] * x + R[i, 1] * y) + R[i, 2] * z   # float32 throughout
    return out


def voxel_keys(points, leaf: float) -> np.ndarray:
    """Integer voxel of every point: floor(float32(p / leaf))."""
    p = np.asarray(points, np.float32).reshape(-1, 3)
    return np.floor(p / np.float32(leaf)).astype(np.int64)


def voxel_count(points, leaf: float) -> int:
    """Number of occupied voxels at this leaf."""
    keys = voxel_keys(points, leaf)
    return len(np.unique(keys, axis=0)) if len(keys) else 0


def voxel_downsample(points, leaf: float) -> np.ndarray:
    """The voxel-grid filter: one mean point per occupied voxel, voxels in
    the order of their first point."""
    p = np.asarray(points, np.float32).reshape(-1, 3)
    if not leaf >= MIN_LEAF:
        raise ValueError("leaf must be at least 2^-10 m")
    if len(p) and not np.all(np.abs(p) < COORD_LIMIT):
        raise ValueError("coordinates must be below 1024 m in magnitude")
    keys = voxel_keys(p, leaf)
    fixed = np.rint(p.astype(np.float64) * FIX_SCALE).astype(np.int64)
    first, sums, counts = {}, [], []
    for i in range(len(p)):
        kk = (int(keys[i, 0]), int(keys[i, 1]), int(keys[i, 2]))
        j = first.get(kk)
        if j is None:
            j = first[kk] = len(sums)
            sums.append([0, 0, 0])
            counts.append(0)
        for a in range(3):
            sums[j][a] += int(fixed[i, a])
        counts[j] += 1
    out = np.empty((len(sums), 3), np.float32)
    for j in range(len(sums)):
        for a in range(3):
            out[j, a] = np.float32(float(sums[j][a]) / counts[j] / FIX_SCALE)
    return out


def choose_leaf(points, target_points: int) -> float:
    """The leaf of the target-size reading (24 float bisection steps)."""
    p = np.asarray(points, np.float32).reshape(-1, 3)
    if len(p) == 0:
        return 1.0
    ext = np.float32(max(float(p[:, a].max() - p[:, a].min()) for a in range(3)))
    lo = np.float32(2.0 ** -10)
    hi = np.float32(max(np.float32(2.0) * ext, np.float32(1.0)))
    for _ in range(BISECT_STEPS):
        mid = np.float32((lo + hi) * np.float32(0.5))
        if voxel_count(p, float(mid)) > target_points:
            lo = mid
        else:
            hi = mid
    return float(hi)


def preprocess(points, gravity=None, leaf: float = 0.0, target_points: int = 0):
    """Gravity alignment (if a reading is given), then the voxel-grid filter
    (at `leaf`, or at the leaf chosen for `target_points`).  Returns
    (points, leaf used or 0)."""
    p = np.asarray(points, np.float32).reshape(-1, 3)
    if gravity is not None and np.any(np.asarray(gravity) != 0):
        p = gravity_align(p, gravity)
    if target_points > 0:
        leaf = choose_leaf(p, target_points)
    if leaf > 0:
        return voxel_downsample(p, leaf), float(np.float32(leaf))
    return p.copy(), 0.0
