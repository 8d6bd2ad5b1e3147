"""Parity of the HIP library with the CPU oracle, through the C ABI.

Integer results (voxel sets, node scores, leaf indices, node counters) must be
bit-identical.  Inputs are the seeded synthetic scenes of `synth`.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2310_10023_amd as bbs
from paper_2310_10023_amd import proposal
import synth

pytestmark = pytest.mark.gpu

RESULT_KEYS = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
               "initial_size", "initial_kept")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def room():
    s = synth.room_scene(0)
    return s, bbs.Map(s.points, 0.5, 4), oracle.Map(s.points, 0.5, 4)


def sorted_rows(a):
    a = np.asarray(a, np.int32).reshape(-1, 3)
    return a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))]


# ------------------------------------------------------------------ map (Sec. III-C)

@pytest.mark.parametrize("r,levels,dilate", [(0.5, 4, True), (0.3, 3, True), (1.0, 2, False)])
def test_map_levels_equal_oracle(r, levels, dilate):
    say("map parity", r, levels, dilate)
    s = synth.room_scene(1)
    g = bbs.Map(s.points, r, levels, dilate_leaf=dilate)
    o = oracle.Map(s.points, r, levels, dilate_leaf=dilate)
    info = g.info()
    for l in range(levels + 1):
        got = g.dump_level(l)
        want = sorted_rows(o.level_keys(l))
        assert info["voxels"][l] == len(want)
        np.testing.assert_array_equal(got, want)


def test_map_membership_probes(room):
    say("membership")
    _, g, o = room
    rng = np.random.default_rng(0)
    for l in range(5):
        keys = o.level_keys(l)
        hits = g.contains(l, keys)
        assert hits.all()
        q = rng.integers(keys.min(0) - 3, keys.max(0) + 4, size=(20000, 3)).astype(np.int32)
        want = np.array([o.contains(l, *v) for v in q.tolist()])
        np.testing.assert_array_equal(g.contains(l, q), want)
        assert (~want).sum() > 1000


def test_map_from_device_tensor():
    import torch
    say("map from device tensor")
    s = synth.tiny_scene(3, n_map=700)
    t = torch.from_numpy(s.points).cuda()
    g = bbs.Map(t, 0.25, 3)
    o = oracle.Map(s.points, 0.25, 3)
    for l in range(4):
        np.testing.assert_array_equal(g.dump_level(l), sorted_rows(o.level_keys(l)))


# ------------------------------------------------------------------ score (Eq. (12), Sec. III-C)

def random_nodes(s, rng, n, levels):
    rows = []
    for _ in range(n):
        l = int(rng.integers(0, levels + 1))
        t = [int(rng.integers((s.lo[i] >> l) - 1, (s.hi[i] >> l) + 2)) for i in range(3)]
        a = [int(rng.integers(0, s.n(ax, l))) for ax in range(3)]
        rows.append([l] + t + a)
    return np.array(rows, np.int32)


@pytest.mark.parametrize("k", [1, 37, 256, 2000, 2333])
def test_scores_equal_oracle_room(room, k):
    say("scores room k =", k)
    scene, g, o = room
    sc = synth.scan_scene(scene, 11 + k, k, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    s = oracle.Search(o, sc.points, lo, hi)
    nodes = random_nodes(s, np.random.default_rng(k), 3000, 4)
    want = s.score_nodes(nodes, threads=8)
    got = bbs.score_nodes(g, sc.points, lo, hi, nodes)
    np.testing.assert_array_equal(got, want)
    assert all(g.info()["dense"])          # the room's levels are read from dense grids


def test_scores_hash_layout_equal_oracle():
    """Two copies of the room 900 m apart: the bounding boxes of the fine
    levels are mostly empty, so those levels get no dense grid and their
    lookups probe the hash table (the coarsest level is small enough for a
    grid); scores still equal the oracle's."""
    say("scores hash layout")
    room = synth.room_scene(0)
    both = np.concatenate([room.points, room.points + np.array([900.0, 0.0, 0.0], np.float32)])
    g = bbs.Map(both, 0.5, 4)
    assert not any(g.info()["dense"][:4])
    o = oracle.Map(both, 0.5, 4)
    sc = synth.scan_scene(room, 7, 1500, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    s = oracle.Search(o, sc.points, lo, hi)
    nodes = random_nodes(s, np.random.default_rng(21), 3000, 4)
    np.testing.assert_array_equal(bbs.score_nodes(g, sc.points, lo, hi, nodes), s.score_nodes(nodes, threads=8))


def test_scores_non_power_of_two_voxel():
    say("scores r = 0.3")
    scene = synth.room_scene(2)
    g = bbs.Map(scene.points, 0.3, 3)
    o = oracle.Map(scene.points, 0.3, 3)
    sc = synth.scan_scene(scene, 5, 1500, z=1.5, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    s = oracle.Search(o, sc.points, lo, hi)
    nodes = random_nodes(s, np.random.default_rng(9), 2000, 3)
    np.testing.assert_array_equal(bbs.score_nodes(g, sc.points, lo, hi, nodes), s.score_nodes(nodes, threads=8))


def test_scores_translation_only_grid(room):
    say("scores translation-only")
    scene, g, o = room
    sc = synth.scan_scene(scene, 4, 1000, z=1.5, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    s = oracle.Search(o, sc.points, lo, hi, translation_only=True)
    nodes = random_nodes(s, np.random.default_rng(4), 2000, 4)
    np.testing.assert_array_equal(bbs.score_nodes(g, sc.points, lo, hi, nodes, translation_only=True),
                                  s.score_nodes(nodes, threads=8))


# ------------------------------------------------------------------ localize (Alg. 2)

def compare(got, want):
    for key in RESULT_KEYS:
        assert got[key] == want[key], (key, got[key], want[key])
    if want["found"]:
        # pose = r * leaf and the leaf-level angular cell centres, rounded to float32
        np.testing.assert_array_equal(np.float32(got["pose"]), np.float32(want["pose"]))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("batch", [10000, 64])
def test_localize_room_equals_oracle(room, seed, batch):
    say("localize room", seed, batch)
    scene, g, o = room
    sc = synth.scan_scene(scene, seed, 2000, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=batch, threads=8)
    got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch)
    compare(got, want)


@pytest.mark.parametrize("batch", [1, 7, 333])
@pytest.mark.parametrize("translation_only", [False, True])
def test_localize_tiny_batches_and_modes(batch, translation_only):
    say("localize tiny", batch, translation_only)
    scene = synth.tiny_scene(2, n_map=600)
    g = bbs.Map(scene.points, 0.5, 3)
    o = oracle.Map(scene.points, 0.5, 3)
    sc = synth.scan_scene(scene, 2, 300, z=1.0, rp_deg=2.0, n_beams=16, n_az=256, max_range=12.0)
    rp = math.radians(2.0)
    lo = np.array([-3, -3, 0.5, -rp, -rp, 0], np.float32)
    hi = np.array([3, 3, 1.5, rp, rp, 2 * math.pi], np.float32)
    for T in (0, 150, 280, 301):
        want = oracle.Search(o, sc.points, lo, hi, translation_only=translation_only).localize(T, batch=batch,
                                                                                             threads=8)
        got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, translation_only=translation_only)
        compare(got, want)


def test_localize_single_level_and_single_point():
    say("localize l_max = 0, k = 1")
    scene = synth.tiny_scene(1, n_map=400)
    g = bbs.Map(scene.points, 0.5, 0)
    o = oracle.Map(scene.points, 0.5, 0)
    lo = np.array([-2, -2, 1, 0, 0, 0], np.float32)
    hi = np.array([2, 2, 1, 0, 0, 2 * math.pi], np.float32)
    for k in (1, 50):
        sc = synth.scan_scene(scene, 7, k, z=1.0, rp_deg=0.5, n_beams=8, n_az=128, max_range=12.0)
        for T in (0, k):
            want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=16, threads=4)
            compare(bbs.localize(g, sc.points, lo, hi, T, batch_size=16), want)


def test_localize_device_scan_and_determinism(room):
    import torch
    say("localize device scan, twice")
    scene, g, o = room
    sc = synth.scan_scene(scene, 5, 2000, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=500, threads=8)
    ws = bbs.Workspace()
    dev = torch.from_numpy(sc.points).cuda()
    a = bbs.localize(g, dev, lo, hi, T, batch_size=500, workspace=ws)
    b = bbs.localize(g, sc.points, lo, hi, T, batch_size=500, workspace=ws)
    compare(a, want)
    compare(b, want)


def test_localize_profile_sampling(room):
    """Timing every launch or every 4th changes nothing in the result; both
    report every scoring launch and a positive duration."""
    say("localize with launch timing")
    scene, g, o = room
    sc = synth.scan_scene(scene, 2, 2000, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=64, threads=8)
    ws = bbs.Workspace()
    runs = [bbs.localize(g, sc.points, lo, hi, T, batch_size=64, workspace=ws, profile=p) for p in (0, 1, 4)]
    for r in runs:
        compare(r, want)
    assert runs[1]["score_launches"] == runs[2]["score_launches"] > 4
    assert runs[1]["score_kernel_ms"] > 0 and runs[2]["score_kernel_ms"] > 0


@pytest.mark.parametrize("batch", [64, 10000])
def test_localize_persistent_equals_oracle(room, batch):
    """The persistent cooperative kernel runs the same schedule."""
    say("localize persistent", batch)
    scene, g, o = room
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    for seed in (0, 3):
        sc = synth.scan_scene(scene, seed, 2000, z=1.5, z_jitter=0.25, rp_deg=2.0)
        want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=batch, threads=8)
        got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, persistent=True)
        compare(got, want)
        assert got["persistent_used"] == 1


def test_localize_graph_equals_oracle(room):
    """Graph-captured iterations, replayed several times per search."""
    say("localize graph")
    scene, g, o = room
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    for seed in (1, 2):
        sc = synth.scan_scene(scene, seed, 2000, z=1.5, z_jitter=0.25, rp_deg=2.0)
        want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=64, threads=8)
        compare(bbs.localize(g, sc.points, lo, hi, T, batch_size=64, graph=True), want)


def test_autotune_returns_a_measured_pair(room):
    say("autotune")
    scene, g, _ = room
    lo, hi = synth.search_range_room()
    scans = [synth.scan_scene(scene, 60 + i, 2000, z=1.5, rp_deg=2.0).points for i in range(2)]
    best, allv = bbs.autotune(g, scans, lo, hi, [synth.threshold_95(2000)] * 2, [1000, 10000], [512, 4096])
    assert len(allv) == 4 and all(e["ms"] > 0 for e in allv)
    assert best["ms"] == min(e["ms"] for e in allv)
    assert sorted((e["batch_size"], e["score_items"]) for e in allv) == [(1000, 512), (1000, 4096), (10000, 512),
                                                                         (10000, 4096)]
    # the pick is a configuration like any other: the oracle's result at its batch size
    _, _, o = room
    for sc in scans:
        want = oracle.Search(o, sc, lo, hi).localize(synth.threshold_95(2000), batch=best["batch_size"], threads=8)
        compare(bbs.localize(g, sc, lo, hi, synth.threshold_95(2000), batch_size=best["batch_size"],
                             score_items=best["score_items"]), want)


@pytest.mark.parametrize("items", [1, 300, 20000])
def test_localize_score_tiling_does_not_change_results(room, items):
    say("score_items", items)
    scene, g, o = room
    lo, hi = synth.search_range_room()
    sc = synth.scan_scene(scene, 8, 2500, z=1.5, z_jitter=0.25, rp_deg=2.0)
    T = synth.threshold_95(2500)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=3000, threads=8)
    compare(bbs.localize(g, sc.points, lo, hi, T, batch_size=3000, score_items=items), want)


def test_localize_errors(room):
    say("error paths")
    scene, g, _ = room
    sc = synth.scan_scene(scene, 0, 500, z=1.5, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    bad = sc.points.copy()
    bad[3, 1] = np.nan
    with pytest.raises(bbs.BbsError) as e:
        bbs.localize(g, bad, lo, hi, 400)
    assert e.value.status == -1
    with pytest.raises(bbs.BbsError):
        bbs.localize(g, sc.points, hi, lo, 400)
    # a queue that cannot hold the initial set
    ws = bbs.Workspace(max_queue_nodes=16)
    with pytest.raises(bbs.BbsError) as e:
        bbs.localize(g, sc.points, lo, hi, 0, workspace=ws)
    assert e.value.status == -4
    # the same workspace still works for a search that fits
    r = bbs.localize(g, sc.points, lo, hi, 501, workspace=ws)
    assert r["found"] == 0 and r["nodes_expanded"] == 0


def test_localize_empty_inputs_are_errors(room):
    say("empty inputs")
    scene, g, _ = room
    lo, hi = synth.search_range_room()
    with pytest.raises(bbs.BbsError) as e:
        bbs.localize(g, np.zeros((0, 3), np.float32), lo, hi, 0)
    assert e.value.status == -1
    with pytest.raises(bbs.BbsError) as e:
        bbs.Map(np.zeros((0, 3), np.float32), 0.5, 2)
    assert e.value.status == -1


def test_localize_scan_off_the_map(room):
    """Every point misses the map: all scores are 0, nothing reaches T = 1."""
    say("scan off the map")
    scene, g, o = room
    sc = synth.scan_scene(scene, 3, 800, z=1.5, rp_deg=2.0)
    far = sc.points + np.array([5000.0, 0.0, 0.0], np.float32)
    lo, hi = synth.search_range_room()
    want = oracle.Search(o, far, lo, hi).localize(1, batch=1000, threads=8)
    got = bbs.localize(g, far, lo, hi, 1, batch_size=1000)
    compare(got, want)
    assert got["found"] == 0 and got["nodes_expanded"] == 0


def test_localize_single_cell_fixed_angles(room):
    """One translation leaf and fixed angles: the search scores one leaf."""
    say("single cell")
    scene, g, o = room
    sc = synth.scan_scene(scene, 9, 1000, z=1.5, rp_deg=0.0)
    p = sc.pose
    cell = np.floor(p[:3] / 0.5) * 0.5
    lo = np.array([cell[0], cell[1], cell[2], 0, 0, p[5]], np.float32)
    hi = np.array([cell[0], cell[1], cell[2], 0, 0, p[5]], np.float32)
    for T in (0, 500, 1001):
        want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=100, threads=4)
        got = bbs.localize(g, sc.points, lo, hi, T, batch_size=100)
        compare(got, want)
    assert want["nodes_scored"] == want["initial_size"]


@pytest.mark.parametrize("batch", [3000, 64000])
def test_localize_ragged_range_negative_yaw(room, batch):
    """Translation bounds off the voxel grid and a yaw range starting below
    zero (the prior's yaw bins wrap), with and without a prior."""
    say("ragged range, batch", batch)
    scene, g, o = room
    sc = synth.scan_scene(scene, 12, 1500, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo = np.array([-9.73, -8.11, 1.07, -0.03, -0.03, -1.3], np.float32)
    hi = np.array([8.41, 9.37, 1.93, 0.03, 0.03, 4.1], np.float32)
    T = int(0.9 * 1500)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=batch, threads=8)
    compare(bbs.localize(g, sc.points, lo, hi, T, batch_size=batch), want)
    prior = np.random.default_rng(12).normal(size=1088).astype(np.float32)
    got = bbs.localize(g, sc.points, lo, hi, T, batch_size=batch, prior=prior, seed_beam=8)
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=batch, threads=8, prior=prior,
                                                        seed_beam=got["seed_beam_used"])
    compare(got, want)
    assert (got["seeded"], got["seed_score"]) == (want["seeded"], want["seed_score"])


@pytest.mark.parametrize("translation_only", [False, True])
@pytest.mark.parametrize("beam", [0, 3, 16, 1000])
def test_localize_with_prior_equals_oracle(room, translation_only, beam):
    """Prior-ordered initial set and seed beam: same schedule as the oracle
    (the oracle runs at the beam width the library reports after clamping)."""
    say("localize prior", translation_only, beam)
    scene, g, o = room
    sc = synth.scan_scene(scene, 21, 1200, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    if translation_only:
        lo = lo.copy()
        hi = hi.copy()
        lo[:2], hi[:2] = sc.pose[:2] - 2.0, sc.pose[:2] + 2.0
    T = synth.threshold_95(1200)
    prior = np.random.default_rng(3).normal(size=1088).astype(np.float32) * 2
    got = bbs.localize(g, sc.points, lo, hi, T, batch_size=500, translation_only=translation_only, prior=prior,
                       seed_beam=beam)
    assert got["seed_beam_used"] <= min(beam, 64)
    if beam:
        assert got["seed_beam_used"] > 0
    want = oracle.Search(o, sc.points, lo, hi, translation_only=translation_only).localize(
        T, batch=500, threads=8, prior=prior, seed_beam=got["seed_beam_used"])
    compare(got, want)
    assert got["prior_used"] == want["prior_used"] == 1
    assert (got["seeded"], got["seed_score"]) == (want["seeded"], want["seed_score"])


def test_true_pose_prior_seeds_the_incumbent(room):
    """A prior peaked at the scan's true yaw bin and translation cell leads
    the beam to a leaf at or above the threshold."""
    say("true-pose prior")
    scene, g, o = room
    sc = synth.scan_scene(scene, 23, 1500, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(1500)
    prior = np.zeros(1088, np.float32)
    prior[proposal.yaw_bin(sc.pose[5])] = 8.0
    prior[64 + proposal.xy_cell(sc.pose[0], sc.pose[1], lo, hi)] = 8.0
    got = bbs.localize(g, sc.points, lo, hi, T, batch_size=2000, prior=prior, seed_beam=8)
    assert got["seeded"] == 1 and got["seed_score"] >= T
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=2000, threads=8, prior=prior,
                                                         seed_beam=got["seed_beam_used"])
    compare(got, want)


def test_serve_matches_single_queries(room):
    """Concurrent workers on separate streams give the oracle's results."""
    say("serve")
    scene, g, o = room
    lo, hi = synth.search_range_room()
    scans, want = [], []
    for seed in range(6):
        sc = synth.scan_scene(scene, 40 + seed, 1500 + 97 * seed, z=1.5, z_jitter=0.25, rp_deg=2.0)
        scans.append(sc.points)
        want.append(oracle.Search(o, sc.points, lo, hi).localize(synth.threshold_95(len(sc.points)), batch=2000,
                                                                  threads=8))
    arrivals = np.cumsum(np.random.default_rng(0).exponential(0.002, size=6))
    res, t0, t1 = bbs.serve(g, scans, [(lo, hi)] * 6, [synth.threshold_95(len(s)) for s in scans], arrivals,
                            workers=3, batch_size=2000)
    for got, w in zip(res, want):
        compare(got, w)
    assert np.all(t1 >= t0) and np.all(t0 >= arrivals - 1e-6)


def test_serve_with_per_query_priors_matches_single_queries(room):
    """Learned ordering in a stream: each query's own prior (one query
    without) and a seed beam give what a single search with the same prior
    gives; the persistent kernel, which fills the GPU, is refused with more
    than one worker."""
    say("serve, per-query priors")
    scene, g, _ = room
    lo, hi = synth.search_range_room()
    rng = np.random.default_rng(3)
    scans, priors = [], []
    for seed in range(4):
        scans.append(synth.scan_scene(scene, 50 + seed, 1800, z=1.5, z_jitter=0.25, rp_deg=2.0).points)
        priors.append(rng.normal(size=1088).astype(np.float32))
    priors[2] = None
    thr = [synth.threshold_95(len(s)) for s in scans]
    arrivals = np.cumsum(rng.exponential(0.002, size=4))
    res, t0, t1 = bbs.serve(g, scans, [(lo, hi)] * 4, thr, arrivals, workers=2, batch_size=2000, priors=priors,
                            seed_beam=8)
    for sc, p, t, got in zip(scans, priors, thr, res):
        want = bbs.localize(g, sc, lo, hi, t, batch_size=2000, prior=p, seed_beam=8)
        compare(got, want)
        assert got["prior_used"] == (p is not None)
        assert (got["seeded"], got["seed_score"]) == (want["seeded"], want["seed_score"])
    with pytest.raises(bbs.BbsError, match="one worker"):
        bbs.serve(g, scans, [(lo, hi)] * 4, thr, arrivals, workers=2, batch_size=2000, persistent=True)


# ------------------------------------------------------------------ full-size city (sampled parity)

@pytest.fixture(scope="module")
def city():
    c = synth.city_scene(1000)
    say("city map points", len(c.points))
    return c, bbs.Map(c.points, 1.0, 6), oracle.Map(c.points, 1.0, 6)


def test_city_map_and_sampled_scores(city):
    say("city map + sampled scores")
    c, g, o = city
    info = g.info()
    for l in range(7):
        assert info["voxels"][l] == o.level_size(l)
    np.testing.assert_array_equal(g.dump_level(6), sorted_rows(o.level_keys(6)))
    np.testing.assert_array_equal(g.dump_level(0), sorted_rows(o.level_keys(0)))
    sc = synth.scan_scene(c, 0, 10000, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048, voxel=0.5)
    lo, hi = synth.search_range_city()
    s = oracle.Search(o, sc.points, lo, hi)
    nodes = random_nodes(s, np.random.default_rng(1), 1500, 6)
    np.testing.assert_array_equal(bbs.score_nodes(g, sc.points, lo, hi, nodes), s.score_nodes(nodes, threads=16))


def test_city_scores_largest_scan(city):
    """Sampled node scores at the largest scan size of the stream workload
    (30,000 points) on the full city map."""
    say("city scores K = 30000")
    c, g, o = city
    sc = synth.scan_scene(c, 77, 30000, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048, voxel=0.25)
    lo, hi = synth.search_range_city()
    s = oracle.Search(o, sc.points, lo, hi)
    nodes = random_nodes(s, np.random.default_rng(30), 600, 6)
    np.testing.assert_array_equal(bbs.score_nodes(g, sc.points, lo, hi, nodes), s.score_nodes(nodes, threads=16))


def test_city_localize_equals_oracle(city):
    """Full 10k-point city query, plain batched b = 10000, against the oracle."""
    say("city localize seed 0")
    c, g, o = city
    sc = synth.scan_scene(c, 0, 10000, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048, voxel=0.5)
    lo, hi = synth.search_range_city()
    T = synth.threshold_95(10000)
    got = bbs.localize(g, sc.points, lo, hi, T, batch_size=10000)
    say("gpu", {k: got[k] for k in RESULT_KEYS}, got["phase_ms"])
    pers = bbs.localize(g, sc.points, lo, hi, T, batch_size=10000, persistent=True)
    say("gpu persistent", pers["phase_ms"], pers["persistent_used"])
    want = oracle.Search(o, sc.points, lo, hi).localize(T, batch=10000, threads=16)
    compare(got, want)
    compare(pers, want)
