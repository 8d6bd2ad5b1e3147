"""The exact rotational bound on the device (option rot_exact: coarse levels
scored against the map's grown tables) against the oracle's
(`tests/test_oracle_rotbound.py` pins that one): the margins, per-node scores,
whole searches at several batch sizes and loop forms, and the property the
bound buys: a prior and seed beam cannot change the result."""
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


def d_max(points):
    p = np.asarray(points, np.float64)
    return float(np.sqrt(((p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1]) + p[:, 2] * p[:, 2]).max()))


def tiny(seed, k=120, rp_deg=1.0, yaw=1.2, levels=3):
    scene = synth.tiny_scene(seed, n_map=500)
    scan = synth.scan_scene(scene, seed, k, z=1.0, rp_deg=max(rp_deg, 0.5), n_beams=16, n_az=256,
                            max_range=12.0).points
    rp = math.radians(rp_deg)
    lo = np.array([-2, -2, 0.5, -rp, -rp, 0.0], np.float32)
    hi = np.array([2, 2, 1.5, rp, rp, yaw], np.float32)
    need = oracle.Search(oracle.Map(scene.points, 0.5, levels), scan, lo, hi).margins_needed()
    o = oracle.Search(oracle.Map(scene.points, 0.5, levels, margins=need), scan, lo, hi, rot_exact=True)
    g = bbs.Map(scene.points, 0.5, levels, margins=need)
    return scan, lo, hi, need, o, g


@pytest.fixture(scope="module")
def room():
    scene = synth.room_scene(0)
    lo, hi = synth.search_range_room()
    sc = synth.room_query(scene, 0, 2000)
    need = oracle.Search(oracle.Map(scene.points, 0.5, 4), sc.points, lo, hi).margins_needed()
    return scene, lo, hi, need, bbs.Map(scene.points, 0.5, 4, margins=need), \
        oracle.Map(scene.points, 0.5, 4, margins=need)


def test_margins_equal_oracle():
    for seed in range(4):
        scan, lo, hi, need, o, g = tiny(seed)
        assert bbs.rotation_margins(0.5, 3, d_max(scan), lo, hi) == need, seed
    scene = synth.room_scene(0)
    lo, hi = synth.search_range_room()
    for seed in range(3):
        sc = synth.room_query(scene, seed, 2000)
        want = oracle.Search(oracle.Map(scene.points[:2000], 0.5, 4), sc.points, lo, hi).margins_needed()
        assert bbs.rotation_margins(0.5, 4, d_max(sc.points), lo, hi) == want


def test_node_scores_equal_oracle(room):
    scene, lo, hi, need, g, om = room
    sc = synth.room_query(scene, 1, 2000)
    o = oracle.Search(om, sc.points, lo, hi, rot_exact=True)
    rng = np.random.default_rng(2)
    nodes = []
    for level in range(0, 5):
        for _ in range(300):
            nodes.append([level] + [int(rng.integers(o.lo[a] >> level, (o.hi[a] >> level) + 1)) for a in range(3)]
                         + [int(rng.integers(0, o.n(a, level))) for a in range(3)])
    nodes = np.array(nodes, np.int32)
    want = o.score_nodes(nodes, threads=8)
    got = bbs.score_nodes(g, sc.points, lo, hi, nodes, rot_exact=True)
    np.testing.assert_array_equal(got, want)
    plain = bbs.score_nodes(g, sc.points, lo, hi, nodes)
    assert np.all(got >= plain) and np.any(got > plain)


@pytest.mark.parametrize("seed", [0, 1, 3])
def test_tiny_searches_equal_oracle(seed):
    scan, lo, hi, need, o, g = tiny(seed)
    for frac in (0.5, 0.9):
        T = int(math.ceil(frac * len(scan)))
        for b in (1, 7, 64, 10000):
            say("rot exact tiny", seed, frac, b)
            want = o.localize(T, batch=b, threads=8)
            compare(bbs.localize(g, scan, lo, hi, T, batch_size=b, rot_exact=True), want, (seed, frac, b))


def test_room_searches_equal_oracle_in_every_loop_form(room):
    scene, lo, hi, need, g, om = room
    T = synth.threshold_95(2000)
    for seed in (0, 2):
        sc = synth.room_query(scene, seed, 2000)
        want = oracle.Search(om, sc.points, lo, hi, rot_exact=True).localize(T, batch=10000, threads=8)
        say("rot exact room", seed, want["nodes_scored"])
        for kw in ({}, {"persistent": True}, {"graph": True}):
            compare(bbs.localize(g, sc.points, lo, hi, T, rot_exact=True, **kw), want, (seed, kw))


def test_prior_and_beam_cannot_change_the_result(room):
    scene, lo, hi, need, g, om = room
    T = synth.threshold_95(2000)
    rng = np.random.default_rng(4)
    for seed in (1, 3):
        sc = synth.room_query(scene, seed, 2000)
        base = bbs.localize(g, sc.points, lo, hi, T, rot_exact=True)
        for beam in (0, 8, 32):
            r = bbs.localize(g, sc.points, lo, hi, T, rot_exact=True, prior=rng.normal(size=1088), seed_beam=beam)
            assert (r["found"], r["score"], r["leaf"]) == (base["found"], base["score"], base["leaf"]), (seed, beam)


def test_missing_or_small_margins_are_rejected(room):
    scene, lo, hi, need, g, om = room
    sc = synth.room_query(scene, 0, 2000)
    plain_map = bbs.Map(scene.points, 0.5, 4)
    with pytest.raises(bbs.BbsError, match="margin"):
        bbs.localize(plain_map, sc.points, lo, hi, 1900, rot_exact=True)
    small = bbs.Map(scene.points, 0.5, 4, margins=[0] + [max(0, e - 1) for e in need[1:]])
    with pytest.raises(bbs.BbsError, match="margin"):
        bbs.localize(small, sc.points, lo, hi, 1900, rot_exact=True)
    # translation-only grids need no margins
    bbs.localize(plain_map, sc.points, lo, hi, 1900, rot_exact=True, translation_only=True)
