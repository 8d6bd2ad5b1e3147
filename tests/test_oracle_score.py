"""Pins for the oracle's node score, the upper bound of Eq. (12):
score(c) = sum_k H^{c_l}(T_{x_c} s_k).

Two independent pins:
  * hand-worked single-point cases (tests/golden/score_hand.json), which fix
    the dilation direction, the translation x_c = r_l c, the rotation sense and
    the level arithmetic;
  * the literal formula evaluated here with different code: the rotation from
    scipy, the transform and floor((R s + r_l c) / r_l) in double precision, the
    occupancy set from exact rational arithmetic.  Points within 1e-4 voxel of a
    voxel boundary may legitimately round either way in float32 and are
    counted as "either".
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from test_oracle_map import literal_sets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_scores():
    cases = json.load(open(os.path.join(GOLDEN, "score_hand.json")))["cases"]
    for case in cases:
        m = oracle.Map(np.array(case["map"], np.float32), case["r"], case["levels"])
        ang = case["angles"]
        lo = np.array([-50, -50, -50] + ang, np.float32)
        hi = np.array([50, 50, 50] + ang, np.float32)
        s = oracle.Search(m, np.array(case["scan"], np.float32), lo, hi)
        for (level, x, y, z, want) in case["expect"]:
            got = s.score(level, x, y, z, 0, 0, 0)
            assert got == want, (case["name"], level, x, y, z)


def literal_score(sets, scan, r, level, t, angles):
    R = Rotation.from_euler("xyz", angles).as_matrix()
    rl = r * (2 ** level)
    p = (scan.astype(np.float64) @ R.T + rl * np.asarray(t, np.float64)) / rl
    keys = np.floor(p).astype(np.int64)
    amb = np.any(np.abs(p - np.round(p)) < 1e-4, axis=1)
    D = sets[level]
    hit = np.array([tuple(k) in D for k in keys.tolist()])
    return int(hit[~amb].sum()), int(amb.sum())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_score_matches_literal_formula(seed):
    rng = np.random.default_rng(seed)
    scene = synth.tiny_scene(seed, n_map=400)
    r, L = 0.5, 3
    m = oracle.Map(scene.points, r, L)
    sets = literal_sets(scene.points, r, L)
    scan = synth.scan_scene(scene, seed, 300, z=1.0, rp_deg=3.0, n_beams=16, n_az=256, max_range=20.0).points
    rp = math.radians(3.0)
    lo = np.array([-4, -4, 0.5, -rp, -rp, 0.0], np.float32)
    hi = np.array([4, 4, 1.5, rp, rp, 2 * math.pi], np.float32)
    s = oracle.Search(m, scan, lo, hi)
    dmax = float(np.max(np.linalg.norm(scan.astype(np.float64), axis=1)))
    n_amb_total = 0
    for _ in range(60):
        level = int(rng.integers(0, L + 1))
        t = [int(rng.integers(s.lo[i] >> level, (s.hi[i] >> level) + 1)) for i in range(3)]
        idx = [int(rng.integers(0, s.n(ax, level))) for ax in range(3)]
        # cell-centre angles from the closed form of Eq. (2) and Sec. III-D
        delta = 2 * math.asin(r * 2 ** level / (2 * dmax))
        ang = []
        for ax in range(3):
            W = float(hi[3 + ax]) - float(lo[3 + ax])
            n = math.ceil(W / delta) if W > 0 else 1
            assert n == s.n(ax, level)
            ang.append(float(lo[3 + ax]) + (W / n) * (idx[ax] + 0.5))
        want, amb = literal_score(sets, scan, r, level, t, ang)
        got = s.score(level, *t, *idx)
        assert want <= got <= want + amb, (level, t, idx)
        n_amb_total += amb
    assert n_amb_total < 0.01 * 60 * len(scan)


def test_score_bounds_and_duplicates():
    scene = synth.tiny_scene(4, n_map=300)
    m = oracle.Map(scene.points, 0.5, 2)
    scan = synth.scan_scene(scene, 4, 50, z=1.0, rp_deg=1.0, n_beams=8, n_az=128, max_range=20.0).points
    dup = np.concatenate([scan, scan], 0)
    lo = np.array([-3, -3, 1, 0, 0, 0], np.float32)
    hi = np.array([3, 3, 1, 0, 0, 2 * math.pi], np.float32)
    s1 = oracle.Search(m, scan, lo, hi)
    s2 = oracle.Search(m, dup, lo, hi)
    for node in [(0, 0, 0, 2, 0, 0, 5), (1, -1, 1, 1, 0, 0, 7), (2, 0, 0, 0, 0, 0, 3)]:
        a = s1.score(*node)
        assert 0 <= a <= len(scan)
        assert s2.score(*node) == 2 * a          # duplicate points count separately
