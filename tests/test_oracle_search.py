"""Pins for the oracle's batched best-first branch and bound (Alg. 2, Sec. III-E).

  * Exactness: with translation-only branching (Table I, configurations
    (d)-(f)) the bound is valid, so branch and bound must return the full
    search's optimum (Sec. III-B): the argmax of the leaf score with the
    lexicographically smallest leaf on ties, for every batch size b.  The full
    search is an exhaustive scan of all leaves (argmax taken by numpy here).
  * The bound invariant parent >= child, exhaustively on tiny grids, in
    translation-only mode (dilated coarse levels, Sec. III-C).
  * Special cases: l_max = 0 is the full search; a threshold above K finds
    nothing and branches nothing.
  * Known-pose recovery on noise-free scans, and the paper's success criterion
    (2.0 m, 0.05 rad, Sec. IV) on noisy scans of the room.
  * Schedule invariants of the node counters.  The exact counts and pop order
    are pinned on hand-traced instances in test_oracle_schedule.py.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def tiny_case(seed, k=200, translation_only=True, rp_deg=0.0, levels=3, z_w=0.0):
    scene = synth.tiny_scene(seed, n_map=500)
    scan = synth.scan_scene(scene, seed, k, z=1.0, rp_deg=max(rp_deg, 0.5), n_beams=16, n_az=256,
                            max_range=12.0).points
    m = oracle.Map(scene.points, 0.5, levels)
    rp = math.radians(rp_deg)
    lo = np.array([-2, -2, 1.0 - z_w, -rp, -rp, 0.0], np.float32)
    hi = np.array([2, 2, 1.0 + z_w, rp, rp, 2 * math.pi], np.float32)
    return oracle.Search(m, scan, lo, hi, translation_only=translation_only)


def numpy_full_search(s, threshold):
    sc = s.all_leaf_scores(threads=8)
    flat = sc.ravel()
    i = int(np.argmax(flat))               # first maximum in row-major = lexicographic order
    if flat[i] < threshold:
        return None
    idx = np.unravel_index(i, sc.shape)
    leaf = [int(idx[0]) + s.lo[0], int(idx[1]) + s.lo[1], int(idx[2]) + s.lo[2],
            int(idx[3]), int(idx[4]), int(idx[5])]
    return int(flat[i]), leaf


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("frac", [0.0, 0.5, 0.9])
def test_translation_only_bnb_equals_full_search(seed, frac):
    s = tiny_case(seed)
    T = int(math.ceil(frac * s.k))
    want = numpy_full_search(s, T)
    bf = s.bruteforce(T, threads=8)
    if want is None:
        assert bf["found"] == 0
    else:
        assert bf["found"] == 1 and bf["score"] == want[0] and bf["leaf"] == want[1]
    for b in (1, 7, 64, 10000):
        r = s.localize(T, batch=b, threads=8)
        assert r["found"] == bf["found"], b
        if bf["found"]:
            assert r["score"] == bf["score"] and r["leaf"] == bf["leaf"], b


@pytest.mark.parametrize("seed", [0, 4])
def test_depth_first_translation_only_equals_full_search(seed):
    """The depth-first order of Alg. 1 (Table I, DFS) changes only the pop
    order: with the exact bound of translation-only branching it returns the
    full search's optimum too, at every batch size."""
    s = tiny_case(seed, k=150, rp_deg=1.0, z_w=0.5)
    T = int(0.6 * s.k)
    bf = s.bruteforce(T, threads=8)
    for b in (1, 64, 10000):
        r = s.localize(T, batch=b, threads=8, strategy="depth_first")
        assert r["found"] == bf["found"], b
        if bf["found"]:
            assert r["score"] == bf["score"] and r["leaf"] == bf["leaf"], b


def test_depth_first_pops_levels_in_order():
    """Between two flushes nothing is pushed, so the depth-first pops of one
    batch come in (level ascending, score descending) order, and a leaf is
    reached before any pending parent of a higher level is popped."""
    s = tiny_case(1, k=200, translation_only=False, rp_deg=2.0)
    r = s.localize(int(0.5 * s.k), batch=64, threads=8, events_cap=200000, strategy="depth_first")
    assert r["events_total"] <= 200000
    prev = None
    for e in r["events"]:
        if e[0] == "flush":
            prev = None
            continue
        key = (e[1][0], -e[2])
        if prev is not None:
            assert key >= prev, (prev, key)
        prev = key


def test_translation_only_with_z_and_tilt_axes():
    s = tiny_case(5, k=120, rp_deg=2.0, z_w=0.5)
    T = int(0.6 * s.k)
    bf = s.bruteforce(T, threads=8)
    for b in (3, 500):
        r = s.localize(T, batch=b, threads=8)
        assert (r["found"], r["score"], r["leaf"]) == (bf["found"], bf["score"], bf["leaf"])


def all_nodes(s, level):
    out = []
    for x in range(s.lo[0] >> level, (s.hi[0] >> level) + 1):
        for y in range(s.lo[1] >> level, (s.hi[1] >> level) + 1):
            for z in range(s.lo[2] >> level, (s.hi[2] >> level) + 1):
                for a in range(s.n(0, level)):
                    for b in range(s.n(1, level)):
                        for c in range(s.n(2, level)):
                            out.append((level, x, y, z, a, b, c))
    return np.array(out, np.int32)


@pytest.mark.parametrize("seed", [0, 3])
def test_bound_invariant_translation_only(seed):
    """Every child's score is at most its parent's (exact with the dilated map)."""
    s = tiny_case(seed, k=150, rp_deg=1.0, z_w=0.5)
    checked = 0
    for level in range(1, 4):
        nodes = all_nodes(s, level)
        ps = s.score_nodes(nodes, threads=8)
        for nd, p in zip(nodes, ps):
            ch = s.children(nd)
            if len(ch) == 0:
                continue
            cs = s.score_nodes(ch, threads=1)
            assert cs.max() <= p, (nd, p, cs.max())
            checked += len(ch)
    assert checked > 10000


def test_rotational_branching_violations_are_rare():
    """With rotational branching the bound is approximate (Sec. III-D); the
    oracle counts children scoring above their parent."""
    s = tiny_case(1, k=300, translation_only=False, rp_deg=2.0)
    r = s.localize(int(0.5 * s.k), batch=64, threads=8)
    assert r["bound_checks"] > 0
    assert r["bound_violations"] / r["bound_checks"] < 0.05


@pytest.mark.parametrize("translation_only", [False, True])
def test_single_level_is_full_search(translation_only):
    s = tiny_case(2, k=100, translation_only=translation_only, rp_deg=1.0, levels=0)
    for T in (0, 60):
        bf = s.bruteforce(T, threads=8)
        r = s.localize(T, batch=50, threads=8)
        assert (r["found"], r["score"], r["leaf"]) == (bf["found"], bf["score"], bf["leaf"])
        assert r["nodes_expanded"] == 0 and r["flushes"] == 0


def test_threshold_above_k_finds_nothing():
    s = tiny_case(0, k=100, translation_only=False, rp_deg=1.0)
    r = s.localize(s.k + 1, batch=100, threads=8)
    assert r["found"] == 0 and r["nodes_expanded"] == 0 and r["initial_kept"] == 0
    assert r["nodes_scored"] == r["initial_size"] > 0


@pytest.mark.parametrize("b", [1, 10, 333])
def test_schedule_counter_invariants(b):
    s = tiny_case(4, k=150, translation_only=False, rp_deg=2.0)
    r = s.localize(int(0.7 * s.k), batch=b, threads=8, trace_cap=1 << 20)
    sizes = r["flush_sizes"]
    assert r["nodes_scored"] == r["initial_size"] + sum(sizes)
    assert len(sizes) == r["flushes"]
    fan = max(s.a(0, l) * s.a(1, l) * s.a(2, l) * 8 for l in range(1, 4))
    # a flush is triggered by exceeding b, or by the termination rule (queue empty)
    assert all(1 <= n <= b + fan for n in sizes)
    assert sum(n > b for n in sizes) >= len(sizes) - r["nodes_expanded"]
    assert r["bound_checks"] == sum(sizes)


def known_pose_scan(scene, t, angles, radius, n, seed):
    """Map points within `radius` of t, expressed in the frame of pose (t, angles)."""
    rng = np.random.default_rng(seed)
    d = np.linalg.norm(scene.points.astype(np.float64) - t, axis=1)
    cand = np.nonzero(d < radius)[0]
    pts = scene.points[rng.choice(cand, size=n, replace=False)].astype(np.float64)
    R = synth.rotation_zyx(*angles)
    return ((pts - t) @ R).astype(np.float32)    # R^T (m - t), row-vector form


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_noise_free_known_pose_recovery(seed):
    """A noise-free scan taken at a leaf-grid rotation and a translation inside
    a leaf cell scores K at that leaf (dilated leaf level), and translation-only
    branch and bound returns a K-scoring leaf."""
    rng = np.random.default_rng(seed)
    scene = synth.room_scene(seed)
    r, L = 0.5, 3
    m = oracle.Map(scene.points, r, L)
    ti = np.array([rng.integers(-8, 8), rng.integers(-8, 8), 3])
    frac = rng.uniform(0.05, 0.95, size=3)
    t = (ti + frac) * r
    pts_probe = known_pose_scan(scene, t, (0, 0, 0), 9.0, 300, seed)
    lo = np.array([-6, -6, 1.5, 0, 0, 0], np.float32)
    hi = np.array([6, 6, 1.5, 0, 0, 2 * math.pi], np.float32)
    lo[:2] = t[:2] - 2.0
    hi[:2] = t[:2] + 2.0
    probe = oracle.Search(m, pts_probe, lo, hi, translation_only=True)
    # d_max does not depend on the rotation, so the yaw grid is known before the scan is rotated
    iy = int(rng.integers(0, probe.n(2, 0)))
    yaw = float(lo[5]) + probe.dprime(2, 0) * (iy + 0.5)
    scan = known_pose_scan(scene, t, (0, 0, yaw), 9.0, 300, seed)
    s = oracle.Search(m, scan, lo, hi, translation_only=True)
    assert s.n(2, 0) == probe.n(2, 0)
    assert s.score(0, int(ti[0]), int(ti[1]), int(ti[2]), 0, 0, iy) == s.k
    res = s.localize(s.k, batch=1000, threads=8)
    assert res["found"] == 1 and res["score"] == s.k
    assert abs(res["pose"][0] - t[0]) < 2 * r and abs(res["pose"][1] - t[1]) < 2 * r


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_room_success_criterion(seed):
    """Tiny-indoor configuration: noisy 2,000-point scans are localized within
    2.0 m and 0.05 rad (the success criterion of Sec. IV)."""
    scene = synth.room_scene(0)
    m = oracle.Map(scene.points, 0.5, 4)
    sc = synth.scan_scene(scene, seed, 2000, z=1.5, z_jitter=0.25, rp_deg=2.0)
    lo, hi = synth.search_range_room()
    s = oracle.Search(m, sc.points, lo, hi)
    res = s.localize(synth.threshold_95(2000), batch=10000, threads=8)
    assert res["found"] == 1
    err_t = np.linalg.norm(np.array(res["pose"][:3]) - sc.pose[:3])
    R_est = synth.rotation_zyx(*res["pose"][3:])
    R_true = synth.rotation_zyx(*sc.pose[3:])
    err_r = math.acos(max(-1.0, min(1.0, (np.trace(R_est.T @ R_true) - 1) / 2)))
    assert err_t < 2.0 and err_r < 0.05, (err_t, err_r)


# ------------------------------------------------------------------ learned prior (ordering and seed beam)
#
# Not in the paper.  The prior key of a node is the best yaw-bin logit over
# the leaf yaws below it plus the best translation-cell logit over the leaf
# translations below it.  Pins: a leaf's key is the logit pair of its own
# bins (the label binning of the training data); a parent's key is the
# maximum of its children's keys (the leaves below a node are the disjoint
# union of the leaves below its children, and the children are every
# rotation child paired with every translation child); a seed beam wide
# enough to keep every node reaching the threshold finds the exhaustive
# optimum in translation-only mode (the bound is valid there, so every leaf
# at or above the threshold has all its ancestors at or above it too).


def _label_bins(s, leaf):
    """Yaw bin and translation cell of a leaf, the way training labels are
    binned: the leaf's yaw is its cell centre, its translation r * i."""
    two_pi = 2 * math.pi
    g = s.grid
    yaw = g.wmin[2] + g.dprime[2][0] * (leaf[6] + 0.5)
    yb = int(math.floor((yaw % two_pi) / (two_pi / 64))) % 64
    cells = []
    for ax in range(2):
        x = float(np.float32(g.r)) * leaf[1 + ax]
        c = int(math.floor(32 * (x - g.tmin[ax]) / (g.tmax[ax] - g.tmin[ax])))
        cells.append(min(max(c, 0), 31))
    return yb, cells[0] * 32 + cells[1]


@pytest.mark.parametrize("translation_only", [True, False])
def test_prior_key_of_leaf_is_its_bin_logits(translation_only):
    s = tiny_case(4, translation_only=translation_only, rp_deg=2.0, z_w=0.5)
    rng = np.random.default_rng(11)
    prior = rng.normal(size=1088).astype(np.float32)
    g = s.grid
    for _ in range(200):
        leaf = [0] + [int(rng.integers(g.lo[a], g.hi[a] + 1)) for a in range(3)] + \
               [int(rng.integers(0, g.n[a][0])) for a in range(3)]
        yb, cell = _label_bins(s, leaf)
        assert s.prior_key(prior, leaf) == float(prior[yb]) + float(prior[64 + cell])


@pytest.mark.parametrize("translation_only", [True, False])
def test_prior_key_of_parent_is_max_over_children(translation_only):
    s = tiny_case(5, translation_only=translation_only, rp_deg=2.0, z_w=0.5, levels=3)
    prior = np.random.default_rng(12).normal(size=1088).astype(np.float32) * 4
    L = s.grid.levels
    # walk the tree from every top-level cell, checking every expanded node
    frontier = []
    for x in range(s.grid.lo[0] >> L, (s.grid.hi[0] >> L) + 1):
        for y in range(s.grid.lo[1] >> L, (s.grid.hi[1] >> L) + 1):
            for z in range(s.grid.lo[2] >> L, (s.grid.hi[2] >> L) + 1):
                for ig in range(s.n(2, L)):
                    frontier.append([L, x, y, z, 0, 0, ig])
    checked = 0
    rng = np.random.default_rng(0)
    while frontier and checked < 300:
        node = frontier.pop(int(rng.integers(len(frontier))))
        if node[0] == 0:
            continue
        ch = s.children(node)
        assert len(ch) > 0
        kc = max(s.prior_key(prior, c) for c in ch)
        assert s.prior_key(prior, node) == kc
        checked += 1
        frontier.extend(c.tolist() for c in ch[rng.permutation(len(ch))[:3]])
    assert checked >= 50


@pytest.mark.parametrize("beam", [0, 1, 4])
@pytest.mark.parametrize("seed", [0, 2])
def test_prior_keeps_translation_only_result_exact(seed, beam):
    """Ordering ties by a prior and seeding the incumbent by a beam leave the
    translation-only optimum unchanged (pruning stays strict)."""
    s = tiny_case(seed, rp_deg=2.0, z_w=0.5)
    T = int(0.6 * s.k)
    bf = s.bruteforce(T, threads=8)
    prior = np.random.default_rng(seed).normal(size=1088).astype(np.float32) * 3
    r = s.localize(T, batch=64, threads=8, prior=prior, seed_beam=beam)
    assert r["prior_used"] == 1
    assert (r["found"], r["score"], r["leaf"]) == (bf["found"], bf["score"], bf["leaf"])
    if r["seeded"]:
        assert r["seed_score"] <= r["score"]


@pytest.mark.parametrize("seed", [1, 3])
def test_full_width_beam_finds_exhaustive_optimum(seed):
    s = tiny_case(seed, rp_deg=2.0, z_w=0.5)
    T = int(0.6 * s.k)
    bf = s.bruteforce(T, threads=8)
    assert bf["found"] == 1
    prior = np.random.default_rng(seed).normal(size=1088).astype(np.float32)
    r = s.localize(T, batch=64, threads=8, prior=prior, seed_beam=1 << 30)
    assert r["seeded"] == 1 and r["seed_score"] == bf["score"]
    assert (r["score"], r["leaf"]) == (bf["score"], bf["leaf"])


def test_flat_prior_changes_nothing_and_nan_prior_is_ignored():
    s = tiny_case(1, translation_only=False, rp_deg=2.0)
    T = int(0.7 * s.k)
    plain = s.localize(T, batch=100, threads=8)
    flat = s.localize(T, batch=100, threads=8, prior=np.zeros(1088, np.float32))
    nan = np.zeros(1088, np.float32)
    nan[5] = np.nan
    ign = s.localize(T, batch=100, threads=8, prior=nan, seed_beam=4)
    assert flat["prior_used"] == 1 and ign["prior_used"] == 0 and ign["seeded"] == 0
    for key in ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes"):
        assert flat[key] == plain[key] and ign[key] == plain[key], key


def test_seed_beam_counts_and_incumbent():
    s = tiny_case(3, translation_only=True, rp_deg=2.0, z_w=0.5)
    T = int(0.5 * s.k)
    prior = np.random.default_rng(5).normal(size=1088).astype(np.float32)
    a = s.localize(T, batch=64, threads=8, prior=prior, seed_beam=0)
    b = s.localize(T, batch=64, threads=8, prior=prior, seed_beam=2)
    assert b["seeded"] == 1 and T <= b["seed_score"] <= b["score"] == a["score"]
    # the beam expands at most two nodes per level and scores their children
    L = s.grid.levels
    assert L <= b["nodes_expanded"] - a["nodes_expanded"] + 2 * L
    assert b["nodes_scored"] > b["initial_size"]
