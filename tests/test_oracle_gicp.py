"""Pins of the refinement oracle (voxelized GICP after the search; readings
in `oracle/gicp.py`)."""
import math

import numpy as np
import pytest

import synth
from oracle import gicp


def test_regularized_covariance_is_plane_to_plane():
    rng = np.random.default_rng(0)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    u = np.cross(n, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    pts = rng.normal(size=(200, 2)) @ np.stack([u, v]) * 0.3 + 0.001 * rng.normal(size=(200, 1)) * n
    C = gicp.regularize(np.cov(pts.T, bias=True))
    w, U = np.linalg.eigh(C)
    np.testing.assert_allclose(w, [1e-3, 1.0, 1.0], atol=1e-12)
    assert abs(abs(U[:, 0] @ n) - 1) < 1e-4          # the normal keeps the small eigenvalue


def test_voxel_distributions_hand_worked():
    # four points in voxel (0, 0, 0) of edge 1 (mean (0.5, 0.5, 0)), one alone in (2, 0, 0)
    pts = np.array([[0.25, 0.25, 0], [0.75, 0.25, 0], [0.25, 0.75, 0], [0.75, 0.75, 0], [2.5, 0.5, 0.5]],
                   np.float32)
    keys, mu, C = gicp.voxel_distributions(pts, 1.0, 4)
    np.testing.assert_array_equal(keys, [[0, 0, 0]])
    np.testing.assert_allclose(mu, [[0.5, 0.5, 0.0]])
    # points spread in x and y only: the normal is z
    np.testing.assert_allclose(C[0], np.diag([1.0, 1.0, 1e-3]), atol=1e-12)


def test_pairing_takes_the_nearest_mean_within_one_edge():
    # binary fractions: means exactly (0.5, 0.5, 0) and (1.5, 0.5, 0.875); edge 1
    pts = np.array([[x, y, 0.0] for x in (0.125, 0.375, 0.625, 0.875) for y in (0.25, 0.75)] +
                   [[x + 1, y, 0.875] for x in (0.125, 0.375, 0.625, 0.875) for y in (0.25, 0.75)], np.float32)
    target = gicp.voxel_distributions(pts, 1.0, 4)
    np.testing.assert_array_equal(target[1], [[0.5, 0.5, 0.0], [1.5, 0.5, 0.875]])
    q = np.array([[0.9, 0.5, 0.0],      # in voxel (0,0,0), nearer its own mean
                  [1.02, 0.5, 0.1],     # in voxel (1,0,0), but (0,0,0)'s mean is nearer
                  [1.3, 0.5, 0.7],      # in voxel (1,0,0), nearer its own mean
                  [3.0, 0.5, 0.0],      # no mean within one edge
                  [1.0, 0.5, 0.4375]])  # equidistant: the first offset in order, voxel (0,0,0)
    np.testing.assert_array_equal(gicp.correspond(target, q, 1.0), [0, 0, 1, -1, 0])


def test_gradient_equals_finite_differences_of_the_frozen_cost():
    """g is half the gradient of sum r^T Omega r with Omega and the voxel
    associations held fixed (the Gauss-Newton linearization)."""
    scene = synth.room_scene(0)
    sc = synth.room_query(scene, 1, 1500)
    target = gicp.voxel_distributions(scene.points, 1.0, 5)
    pts, covs = gicp.scan_covariances(sc.points, 1.0, 5)
    R = synth.rotation_zyx(*sc.pose[3:])
    t = sc.pose[:3] + np.array([0.05, -0.04, 0.02])
    H, g, cost, n = gicp.linearize(target, pts, covs, R, t, 1.0)
    assert n > 500
    j = gicp.correspond(target, pts @ R.T + t, 1.0)
    assoc = [(p, target[1][k], np.linalg.inv(target[2][k] + R @ C @ R.T)) for p, C, k in zip(pts, covs, j) if k >= 0]
    assert len(assoc) == n

    def frozen(dx):
        E = gicp.so3_exp(dx[:3])
        s = 0.0
        for p, mu, Om in assoc:
            r = mu - (E @ (R @ p + t) + dx[3:])
            s += r @ Om @ r
        return s

    for i in range(6):
        e = np.zeros(6)
        e[i] = 1e-6
        fd = (frozen(e) - frozen(-e)) / 2e-6
        assert abs(fd - 2 * g[i]) < 1e-4 * max(1.0, abs(fd)), (i, fd, 2 * g[i])
    np.testing.assert_allclose(frozen(np.zeros(6)), cost, rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_recovers_a_known_offset(seed):
    """Noise-free: the scan is a subset of the target's own points seen from a
    known pose; GICP from a 0.3 m / 0.02 rad offset returns to it."""
    scene = synth.room_scene(0)
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(scene.points), 20000, replace=False)
    world = scene.points[idx].astype(np.float64)
    R_true = synth.rotation_zyx(0.01, -0.015, 0.7)
    t_true = np.array([1.0, -2.0, 1.5])
    scan = ((world - t_true) @ R_true).astype(np.float32)     # p = R^T (w - t)
    R0 = synth.rotation_zyx(0.01 + 0.01, -0.015, 0.7 + 0.02)
    t0 = t_true + np.array([0.3, -0.2, 0.1])
    R, t, info = gicp.refine(scene.points, scan, R0, t0, voxel=1.0, min_points=5, max_iterations=30)
    ang = math.acos(min(1.0, (np.trace(R.T @ R_true) - 1) / 2))
    assert np.linalg.norm(t - t_true) < 0.02 and ang < 0.002, (t - t_true, ang, info)
    assert info["pairs"] > 15000 and info["converged"]
