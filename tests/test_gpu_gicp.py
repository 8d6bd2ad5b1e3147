"""Pose refinement on the device (bbs_gicp_*) against the oracle
(`oracle/gicp.py`): one Gauss-Newton linearization, whole refinements, a
known offset recovered, and the search's poses refined on the room.

Tolerances: both sides sum in double, in different orders (device atomics
and workgroup partials, numpy's pairwise sums) and invert 3 x 3 and 6 x 6
systems differently, so H, g and the cost agree to about 1e-12 relative; the
pairing (an integer decision) is the same whenever no transformed point lies
within rounding of a voxel face or of two equidistant means, which the
parity inputs avoid by construction of noise (checked: equal pair counts).
Poses after refinement agree to 1e-8 m and 1e-9 per rotation entry."""
import math
import sys

import numpy as np
import pytest

import paper_2310_10023_amd as bbs
import synth
from oracle import gicp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ang(Ra, Rb):
    return math.acos(max(-1.0, min(1.0, (np.trace(Ra.T @ Rb) - 1) / 2)))


@pytest.fixture(scope="module")
def room():
    scene = synth.room_scene(0)
    return scene, bbs.GicpTarget(scene.points, 1.0, 5), gicp.voxel_distributions(scene.points, 1.0, 5)


def test_linearization_equals_oracle(room):
    scene, tg, ot = room
    for seed in range(3):
        sc = synth.room_query(scene, seed, 2000)
        R = synth.rotation_zyx(*sc.pose[3:]) @ synth.rotation_zyx(0.004, -0.003, 0.01)
        t = sc.pose[:3] + np.array([0.08, -0.05, 0.03])
        pts, covs = gicp.scan_covariances(sc.points, 1.0, 5)
        Hw, gw, cw, nw = gicp.linearize(ot, pts, covs, R, t, 1.0)
        H, g, c, n = tg.linearize(sc.points, R, t, 5)
        say("linearize", seed, n, nw, c, cw)
        assert n == nw and n > 500
        np.testing.assert_allclose(H, Hw, rtol=1e-9, atol=1e-9 * np.abs(Hw).max())
        np.testing.assert_allclose(g, gw, rtol=1e-9, atol=1e-9 * np.abs(gw).max())
        assert abs(c - cw) <= 1e-9 * cw


def test_refinement_equals_oracle(room):
    scene, tg, ot = room
    for seed in (3, 4):
        sc = synth.room_query(scene, seed, 2000)
        R0 = synth.rotation_zyx(*sc.pose[3:]) @ synth.rotation_zyx(0.01, 0.0, -0.02)
        t0 = sc.pose[:3] + np.array([0.2, 0.1, -0.05])
        Rw, tw, iw = gicp.refine(scene.points, sc.points, R0, t0, voxel=1.0, min_points=5, max_iterations=15)
        R, t, info = tg.refine(sc.points, R0, t0, max_iterations=15, min_points=5)
        say("refine", seed, info, iw)
        assert info["iterations"] == iw["iterations"] and info["converged"] == iw["converged"]
        assert info["pairs"] == iw["pairs"]
        np.testing.assert_allclose(t, tw, atol=1e-8)
        np.testing.assert_allclose(R, Rw, atol=1e-9)


def test_recovers_a_known_offset_from_a_device_scan(room):
    import torch
    scene, tg, ot = room
    rng = np.random.default_rng(1)
    world = scene.points[rng.choice(len(scene.points), 20000, replace=False)].astype(np.float64)
    R_true = synth.rotation_zyx(0.01, -0.015, 0.7)
    t_true = np.array([1.0, -2.0, 1.5])
    scan = ((world - t_true) @ R_true).astype(np.float32)
    R0 = synth.rotation_zyx(0.02, -0.015, 0.72)
    t0 = t_true + np.array([0.3, -0.2, 0.1])
    R, t, info = tg.refine(torch.from_numpy(scan).cuda(), R0, t0, max_iterations=30)
    assert np.linalg.norm(t - t_true) < 0.02 and ang(R, R_true) < 0.002 and info["converged"], (t - t_true, info)


def test_search_then_refine_on_the_room(room):
    """The search returns a leaf-cell corner (0.5 m grid); refinement moves it
    to within a few centimetres of the true pose."""
    scene, tg, ot = room
    g = bbs.Map(scene.points, 0.5, 4)
    lo, hi = synth.search_range_room()
    before, after = [], []
    for seed in range(6):
        sc = synth.room_query(scene, seed, 2000)
        r = bbs.localize(g, sc.points, lo, hi, synth.threshold_95(2000))
        assert r["found"]
        R0 = synth.rotation_zyx(*r["pose"][3:])
        t0 = np.asarray(r["pose"][:3], np.float64)
        R, t, info = tg.refine(sc.points, R0, t0, max_iterations=30)
        before.append(np.linalg.norm(t0 - sc.pose[:3]))
        after.append(np.linalg.norm(t - sc.pose[:3]))
        say("search+refine", seed, before[-1], after[-1], info)
    assert np.median(after) < 0.05 and np.median(after) < 0.5 * np.median(before)


def test_error_paths(room):
    import ctypes as C
    scene, tg, ot = room
    L = bbs.lib()
    h = C.c_void_p()
    pts = np.zeros((10, 3), np.float32)
    assert L.bbs_gicp_target_create(pts.ctypes.data, 10, 0, 0.0, 5, None, C.byref(h)) == -1
    assert L.bbs_gicp_target_create(pts.ctypes.data, 10, 0, 1.0, 3, None, C.byref(h)) == -1
    bad = np.array([[np.nan, 0, 0]] * 10, np.float32)
    assert L.bbs_gicp_target_create(bad.ctypes.data, 10, 0, 1.0, 5, None, C.byref(h)) == -1
    with pytest.raises(bbs.BbsError):
        tg.refine(np.zeros((4, 3), np.float32), np.eye(3), np.zeros(3), max_iterations=-1)
