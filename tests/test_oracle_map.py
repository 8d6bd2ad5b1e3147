"""Pins for the oracle's multi-resolution voxel map (Sec. III-C).

The map's level-l set is pinned against the paper's definition written out
independently here: the occupied voxel of a map point m at level l is
floor(m / r_l) with r_l = 2^l r, computed in exact rational arithmetic, and the
dilated set adds v - j for every j in {0,1}^3.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
import synth


def literal_sets(points, r, levels, dilate_leaf=True):
    """D_l by the definition: exact floor(m / (2^l r)), then v - j, j in {0,1}^3."""
    rq = Fraction(float(np.float32(r)))
    out = []
    for l in range(levels + 1):
        rl = rq * (2 ** l)
        occ = set()
        for p in points:
            occ.add(tuple(math.floor(Fraction(float(c)) / rl) for c in p))
        if l == 0 and not dilate_leaf:
            out.append(occ)
            continue
        d = set()
        for (x, y, z) in occ:
            for jx in (0, 1):
                for jy in (0, 1):
                    for jz in (0, 1):
                        d.add((x - jx, y - jy, z - jz))
        out.append(d)
    return out


def random_points(seed, n, scale):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-scale, scale, size=(n, 3)).astype(np.float32)
    # put some points exactly on voxel boundaries (multiples of 0.25) and at zero
    k = n // 4
    p[:k] = (np.round(p[:k] * 4) / 4).astype(np.float32)
    p[k] = 0.0
    p[k + 1] = (-0.0, -0.5, 0.5)
    return p


@pytest.mark.parametrize("r", [0.5, 1.0, 0.25])
@pytest.mark.parametrize("seed", [0, 1])
def test_levels_match_definition(r, seed):
    pts = random_points(seed, 300, 9.0)
    m = oracle.Map(pts, r, 4)
    ref = literal_sets(pts, r, 4)
    for l in range(5):
        got = {tuple(v) for v in m.level_keys(l).tolist()}
        assert got == ref[l], f"level {l}"


def test_undilated_leaf_level():
    pts = random_points(3, 200, 5.0)
    m = oracle.Map(pts, 0.5, 2, dilate_leaf=False)
    ref = literal_sets(pts, 0.5, 2, dilate_leaf=False)
    for l in range(3):
        assert {tuple(v) for v in m.level_keys(l).tolist()} == ref[l]


def test_non_power_of_two_voxel_away_from_edges():
    # with r = 0.3 the float division differs from the exact one only next to a
    # voxel boundary: keep points at least 1e-3 voxel away from any boundary
    rng = np.random.default_rng(7)
    pts = rng.uniform(-20, 20, size=(2000, 3)).astype(np.float32)
    q = pts.astype(np.float64) / float(np.float32(0.3))
    keep = np.all(np.abs(q - np.round(q)) > 1e-3, axis=1)
    pts = pts[keep][:300]
    m = oracle.Map(pts, 0.3, 3)
    ref = literal_sets(pts, 0.3, 3)
    for l in range(4):
        assert {tuple(v) for v in m.level_keys(l).tolist()} == ref[l]


def test_nesting_and_dilation_properties():
    s = synth.room_scene(0)
    m = oracle.Map(s.points, 0.5, 4)
    prev = None
    for l in range(5):
        keys = m.level_keys(l)
        ks = {tuple(v) for v in keys.tolist()}
        if prev is not None:
            # the parent level holds floor(w / 2) of every dilated child key w:
            # w = u - j with u occupied gives floor(w / 2) in {U - 1, U}, U = floor(u / 2)
            par = {(x >> 1, y >> 1, z >> 1) for (x, y, z) in prev}
            assert par <= ks
        prev = ks
        # membership queries agree with the dump
        for v in keys[:: max(1, len(keys) // 200)]:
            assert m.contains(l, *v)
    rng = np.random.default_rng(0)
    ks0 = {tuple(v) for v in m.level_keys(0).tolist()}
    miss = 0
    for v in rng.integers(-40, 40, size=(2000, 3)):
        t = tuple(int(a) for a in v)
        assert m.contains(0, *t) == (t in ks0)
        miss += t not in ks0
    assert miss > 100


def test_invalid_map_arguments():
    pts = np.zeros((4, 3), np.float32)
    with pytest.raises(oracle.OracleError):
        oracle.Map(pts, 0.0, 2)
    with pytest.raises(oracle.OracleError):
        oracle.Map(pts, 1.0, 16)
    bad = pts.copy()
    bad[1, 2] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.Map(bad, 1.0, 2)
