"""The nested angular grid (option nested_angles) on the device against the
oracle's (`orc_grid_nest`, pinned in tests/test_oracle_nested.py): whole
searches on the room and tiny scenes in both branching modes, per-node
scores, the exact rotational bound's margins on it, and exact searches."""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2310_10023_amd as bbs
import synth

pytestmark = pytest.mark.gpu

RESULT_KEYS = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
               "initial_size", "initial_kept")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(got, want, label=""):
    for key in RESULT_KEYS:
        assert got[key] == want[key], (label, key, got[key], want[key])
    if want["found"]:
        np.testing.assert_array_equal(np.float32(got["pose"]), np.float32(want["pose"]), err_msg=str(label))


@pytest.fixture(scope="module")
def room():
    scene = synth.room_scene(0)
    return scene, bbs.Map(scene.points, 0.5, 4), oracle.Map(scene.points, 0.5, 4)


@pytest.mark.parametrize("batch", [64, 10000])
def test_room_equals_oracle(room, batch):
    scene, g, o = room
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    for seed in (0, 1, 2):
        say("nested room", seed, batch)
        sc = synth.room_query(scene, seed, 2000)
        want = oracle.Search(o, sc.points, lo, hi, nested=True).localize(T, batch=batch, threads=8)
        compare(bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, nested_angles=True), want, (seed, batch))


@pytest.mark.parametrize("translation_only", [False, True])
def test_tiny_scenes_equal_oracle(translation_only):
    scene = synth.tiny_scene(3, n_map=600)
    g = bbs.Map(scene.points, 0.5, 3)
    o = oracle.Map(scene.points, 0.5, 3)
    sc = synth.scan_scene(scene, 3, 300, z=1.0, rp_deg=2.0, n_beams=16, n_az=256, max_range=12.0)
    rp = math.radians(2.0)
    lo = np.array([-3, -3, 0.5, -rp, -rp, 0], np.float32)
    hi = np.array([3, 3, 1.5, rp, rp, 2 * math.pi], np.float32)
    for T in (150, 280):
        for b in (1, 7, 333):
            want = oracle.Search(o, sc.points, lo, hi, translation_only=translation_only, nested=True).localize(
                T, batch=b, threads=8)
            got = bbs.localize(g, sc.points, lo, hi, T, batch_size=b, translation_only=translation_only,
                               nested_angles=True)
            compare(got, want, (T, b))


def test_node_scores_and_margins_equal_oracle(room):
    scene, g, o = room
    lo, hi = synth.search_range_room()
    sc = synth.room_query(scene, 3, 2000)
    s = oracle.Search(o, sc.points, lo, hi, nested=True)
    p = np.asarray(sc.points, np.float64)
    dmax = float(np.sqrt(((p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1]) + p[:, 2] * p[:, 2]).max()))
    assert bbs.rotation_margins(0.5, 4, dmax, lo, hi, nested_angles=True) == s.margins_needed()
    rng = np.random.default_rng(5)
    nodes = np.array([[l] + [int(rng.integers(s.lo[a] >> l, (s.hi[a] >> l) + 1)) for a in range(3)]
                      + [int(rng.integers(0, s.n(a, l))) for a in range(3)]
                      for l in range(5) for _ in range(200)], np.int32)
    np.testing.assert_array_equal(bbs.score_nodes(g, sc.points, lo, hi, nodes, nested_angles=True),
                                  s.score_nodes(nodes, threads=8))


def test_exact_bound_on_the_nested_grid_equals_oracle():
    scene = synth.room_scene(0)
    lo, hi = synth.search_range_room()
    sc = synth.room_query(scene, 2, 2000)
    need = oracle.Search(oracle.Map(scene.points[:5000], 0.5, 4), sc.points, lo, hi, nested=True).margins_needed()
    g = bbs.Map(scene.points, 0.5, 4, margins=need)
    o = oracle.Map(scene.points, 0.5, 4, margins=need)
    T = synth.threshold_95(2000)
    want = oracle.Search(o, sc.points, lo, hi, rot_exact=True, nested=True).localize(T, batch=10000, threads=8)
    compare(bbs.localize(g, sc.points, lo, hi, T, rot_exact=True, nested_angles=True), want)
