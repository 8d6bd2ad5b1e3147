"""Scoring groups that share a level and rotation through the scan's voxel
histogram (one lookup per distinct voxel instead of one per point) changes
no score: the whole search equals the oracle's at every setting of the
lowest histogram level, on dense-grid and hash-only levels, and when a
histogram overflows and the run falls back to point-by-point scoring."""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2310_10023_amd as bbs
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
          "initial_size", "initial_kept")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "city_localize.json")


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


@pytest.mark.parametrize("hist_min_level", [-1, 1, 2, 4, 0])
@pytest.mark.parametrize("batch", [10000, 333])
def test_hist_levels_room(room, hist_min_level, batch):
    scene, g, o = room
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    for seed in (0, 6):
        say("hist room", hist_min_level, batch, seed)
        sc = synth.room_query(scene, seed, 2000)
        want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=batch, threads=8)
        got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, hist_min_level=hist_min_level)
        check(got, want, (hist_min_level, batch, seed))


@pytest.mark.parametrize("batch", [1, 7, 64])
@pytest.mark.parametrize("translation_only", [False, True])
def test_hist_tiny_scenes(batch, translation_only):
    say("hist tiny", batch, translation_only)
    scene = synth.tiny_scene(2, n_map=600)
    g = bbs.Map(scene.points, 0.5, 3)
    o = oracle.Map(scene.points, 0.5, 3)
    sc = synth.scan_scene(scene, 2, 300, z=1.0, rp_deg=2.0, n_beams=16, n_az=256, max_range=12.0)
    rp = math.radians(2.0)
    lo = np.array([-3, -3, 0.5, -rp, -rp, 0], np.float32)
    hi = np.array([3, 3, 1.5, rp, rp, 2 * math.pi], np.float32)
    for T in (150, 280):
        want = oracle.Search(o, sc.points, lo, hi, translation_only=translation_only).localize(T, batch=batch,
                                                                                             threads=8)
        got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, translation_only=translation_only,
                           hist_min_level=-1)
        check(got, want, (batch, translation_only, T))


def test_hist_hash_only_levels():
    """Two copies of the room 900 m apart: the fine levels have no dense
    grid, so histogram lookups probe the brick hash table."""
    say("hist hash layout")
    room = synth.room_scene(0)
    both = np.concatenate([room.points, room.points + np.array([900.0, 0.0, 0.0], np.float32)])
    g = bbs.Map(both, 0.5, 4)
    assert not any(g.info()["dense"][:4])
    o = oracle.Map(both, 0.5, 4)
    lo, hi = synth.search_range_room()
    sc = synth.room_query(room, 7, 1500)
    T = synth.threshold_95(1500)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=2000, threads=8)
    check(bbs.localize(g, sc.points, lo, hi, T, batch_size=2000, hist_min_level=-1), want, "hash")


def test_hist_overflow_falls_back_on_the_city():
    """From level 0 up on the city: a 10,000-point scan has more distinct
    level-0 voxels than a histogram holds, so those items score point by
    point; the result is still the oracle's (stored) one."""
    import torch
    with open(GOLDEN) as f:
        doc = json.load(f)
    case = doc["cases"]["bench"]
    want = case["queries"]["0"]
    c = synth.city_scene(1000)
    g = bbs.Map(torch.from_numpy(c.points).cuda(), 1.0, 6)
    sc = synth.city_query(c, 0, case["k"], voxel=case["voxel"])
    lo, hi = np.array(doc["range"]["min"], np.float32), np.array(doc["range"]["max"], np.float32)
    for hml in (-1, 0, 99):
        say("hist city seed 0, hist_min_level", hml)
        got = bbs.localize(g, torch.from_numpy(sc.points).cuda(), lo, hi, case["threshold"], batch_size=case["batch"],
                           hist_min_level=hml)
        check(got, want, ("city", hml))
