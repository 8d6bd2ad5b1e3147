"""Pins of the preprocessing oracle (voxel-grid filter of Sec. IV, gravity
alignment of Sec. III-A / IV-B; readings in `oracle/preprocess.py`)."""
import math

import numpy as np
import pytest

from oracle import preprocess as pp


def test_voxel_filter_hand_worked():
    # binary fractions, so every mean is exact; leaf 1 m
    pts = np.array([[0.125, 0.25, 0.5], [1.5, 0.0, 0.0], [-0.25, 0.0, 0.0], [0.375, 0.75, 0.5],
                    [0.5, 0.5, 0.5], [1.75, 0.5, 0.0]], np.float32)
    out = pp.voxel_downsample(pts, 1.0)
    want = np.array([[np.float32(1.0 / 3.0), 0.5, 0.5],     # voxel (0,0,0): points 0, 3, 4
                     [1.625, 0.25, 0.0],                      # voxel (1,0,0): points 1, 5
                     [-0.25, 0.0, 0.0]], np.float32)          # voxel (-1,0,0)
    np.testing.assert_array_equal(out, want)


def test_voxel_boundaries_floor():
    # a coordinate on a voxel face belongs to the upper voxel; negatives floor down
    keys = pp.voxel_keys(np.array([[1.0, -0.5, -1e-7], [0.49999997, 0.5, 0.0]], np.float32), 0.5)
    np.testing.assert_array_equal(keys, [[2, -1, -1], [0, 1, 0]])


def _grouped_means(pts, leaf):
    """The same filter by a different route: sort voxels, bincount sums."""
    keys = np.floor(pts / np.float32(leaf)).astype(np.int64)
    uniq, first, inv = np.unique(keys, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    fixed = np.rint(pts.astype(np.float64) * 2.0 ** 24)
    cnt = np.bincount(inv)
    means = np.stack([np.bincount(inv, weights=fixed[:, a]) for a in range(3)], 1) / cnt[:, None] / 2.0 ** 24
    order = np.argsort(first)
    return means[order].astype(np.float32)


@pytest.mark.parametrize("leaf", [0.05, 0.3, 1.0, 2.5])
def test_voxel_filter_equals_grouped_means(leaf):
    rng = np.random.default_rng(7)
    pts = (rng.normal(size=(3000, 3)) * np.array([8, 8, 2])).astype(np.float32)
    np.testing.assert_array_equal(pp.voxel_downsample(pts, leaf), _grouped_means(pts, leaf))


def test_voxel_filter_is_order_independent_and_inside_its_voxel():
    rng = np.random.default_rng(3)
    pts = (rng.uniform(-20, 20, size=(4000, 3))).astype(np.float32)
    a = pp.voxel_downsample(pts, 0.7)
    b = pp.voxel_downsample(pts[rng.permutation(len(pts))], 0.7)
    key = lambda x: np.lexsort(x.T[::-1])
    np.testing.assert_array_equal(a[key(a)], b[key(b)])
    k = pp.voxel_keys(a, 0.7)
    lo, hi = k * 0.7, (k + 1) * 0.7
    assert np.all(a >= lo - 1e-5) and np.all(a <= hi + 1e-5)
    assert len(a) == len({tuple(r) for r in pp.voxel_keys(pts, 0.7)})


def test_voxel_filter_rejects_bad_inputs():
    with pytest.raises(ValueError):
        pp.voxel_downsample(np.zeros((2, 3), np.float32), 0.0)
    with pytest.raises(ValueError):
        pp.voxel_downsample(np.array([[1024.0, 0, 0]], np.float32), 1.0)


def rot_x(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def rot_y(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def test_gravity_rotation_special_cases():
    np.testing.assert_array_equal(pp.gravity_rotation([0, 0, 1]), np.eye(3, dtype=np.float32))
    np.testing.assert_array_equal(pp.gravity_rotation([0, 0, 9.81]), np.eye(3, dtype=np.float32))
    np.testing.assert_array_equal(pp.gravity_rotation([0, 0, -1]), np.diag([1, -1, -1]).astype(np.float32))
    pts = np.random.default_rng(1).normal(size=(50, 3)).astype(np.float32)
    np.testing.assert_array_equal(pp.gravity_align(pts, [0, 0, 2]), pts)


@pytest.mark.parametrize("g", [[0.1, -0.2, 0.97], [1, 0, 0], [0.3, 0.4, -0.5], [-2, 5, 1]])
def test_gravity_rotation_is_a_rotation_taking_g_up(g):
    R = pp.gravity_rotation(g).astype(np.float64)
    a = np.asarray(g, np.float64) / np.linalg.norm(g)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-6)
    assert abs(np.linalg.det(R) - 1) < 1e-6
    np.testing.assert_allclose(R @ a, [0, 0, 1], atol=1e-6)
    # the smallest such rotation: its axis is perpendicular to both a and z
    w, v = np.linalg.eig(R)
    axis = np.real(v[:, np.argmin(np.abs(w - 1))])
    assert abs(axis @ a) < 1e-5 and abs(axis[2]) < 1e-5


@pytest.mark.parametrize("roll,pitch", [(0.05, 0.0), (0.0, -0.04), (0.03, 0.02)])
def test_gravity_alignment_undoes_a_tilt(roll, pitch):
    """A sensor tilted by R_t measures up as R_t^T z and sees R_t^T p; the
    alignment restores p (exactly up to a yaw that is zero for a pure roll or
    pitch, and of second order otherwise)."""
    Rt = rot_y(pitch) @ rot_x(roll)
    rng = np.random.default_rng(5)
    pw = rng.uniform(-30, 30, size=(200, 3))
    ps = (pw @ Rt).astype(np.float32)           # rows: R_t^T p
    g = (Rt.T @ np.array([0.0, 0.0, 1.0])).astype(np.float32)
    out = pp.gravity_align(ps, g).astype(np.float64)
    tol = 1e-4 if roll == 0 or pitch == 0 else 0.05
    np.testing.assert_allclose(out, pw, atol=tol)
    # the vertical coordinate is exact for every tilt
    np.testing.assert_allclose(out[:, 2], pw[:, 2], atol=1e-4)


def test_choose_leaf_brackets_the_target():
    # a regular lattice: the voxel count falls monotonically with the leaf
    g = np.arange(0, 20, 0.25, dtype=np.float32)
    pts = np.stack(np.meshgrid(g, g[:40], [0.0], indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    for target in (50, 300, 1000):
        leaf = pp.choose_leaf(pts, target)
        assert pp.voxel_count(pts, leaf) <= target
        assert pp.voxel_count(pts, leaf * (1 - 1e-3)) > target
    out, used = pp.preprocess(pts, target_points=300)
    assert used == pp.choose_leaf(pts, 300) and len(out) <= 300
