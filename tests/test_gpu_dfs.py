"""The depth-first queue order of Alg. 1 (Table I, DFS: deeper levels first,
then higher score) on the device equals the oracle's, node for node."""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2310_10023_amd as bbs
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
          "initial_size", "initial_kept")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(got, want, label):
    for f in FIELDS:
        assert got[f] == want[f], (label, f, got[f], want[f])
    if want["found"]:
        np.testing.assert_array_equal(np.float32(got["pose"]), np.float32(want["pose"]), err_msg=str(label))


@pytest.fixture(scope="module")
def room():
    s = synth.room_scene(0)
    return s, bbs.Map(s.points, 0.5, 4), oracle.Map(s.points, 0.5, 4)


@pytest.mark.parametrize("batch", [64, 500, 10000])
def test_depth_first_room(room, batch):
    scene, g, o = room
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    for seed in (0, 3):
        say("depth first room", batch, seed)
        sc = synth.room_query(scene, seed, 2000)
        want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=batch, threads=8, strategy="depth_first")
        got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, strategy="depth_first")
        check(got, want, (batch, seed))


@pytest.mark.parametrize("batch", [1, 7, 333])
@pytest.mark.parametrize("translation_only", [False, True])
def test_depth_first_tiny_scenes(batch, translation_only):
    say("depth first tiny", batch, translation_only)
    scene = synth.tiny_scene(2, n_map=600)
    g = bbs.Map(scene.points, 0.5, 3)
    o = oracle.Map(scene.points, 0.5, 3)
    sc = synth.scan_scene(scene, 2, 300, z=1.0, rp_deg=2.0, n_beams=16, n_az=256, max_range=12.0)
    rp = math.radians(2.0)
    lo = np.array([-3, -3, 0.5, -rp, -rp, 0], np.float32)
    hi = np.array([3, 3, 1.5, rp, rp, 2 * math.pi], np.float32)
    for T in (0, 150, 280, 301):
        want = oracle.Search(o, sc.points, lo, hi, translation_only=translation_only).localize(
            T, batch=batch, threads=8, strategy="depth_first")
        got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, translation_only=translation_only,
                           strategy="depth_first")
        check(got, want, (batch, translation_only, T))


def test_depth_first_persistent_and_graph(room):
    scene, g, o = room
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    sc = synth.room_query(scene, 1, 2000)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=64, threads=8, strategy="depth_first")
    for kw in ({"persistent": True}, {"graph": True}):
        say("depth first", kw)
        check(bbs.localize(g, sc.points, lo, hi, T, batch_size=64, strategy="depth_first", **kw), want, kw)


def test_strategy_is_validated(room):
    import ctypes as C
    scene, g, _ = room
    lo, hi = synth.search_range_room()
    sc = synth.room_query(scene, 1, 500)
    L = bbs.lib()
    opt = bbs.Options()
    L.bbs_default_options(opt)
    opt.strategy = 2
    res = bbs.Result()
    rng = bbs._range(lo, hi)
    assert L.bbs_localize(g.handle, None, sc.points.ctypes.data, len(sc.points), 0, C.byref(rng), 400, C.byref(opt),
                          C.byref(res)) == -1
    assert b"strategy" in L.bbs_last_error()
