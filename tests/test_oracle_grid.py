"""Pins for the oracle's search grid: Eq. (2), delta'(r_l), the divisions a
(Sec. III-D), the translation index set of Eq. (1), the rotation convention
(Sec. III-A) and the roto-translational branching rule (Sec. III-D)."""
import json
import math
import os
from collections import Counter

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_point_scan(dmax, extra=50, seed=0):
    """A scan whose largest range is exactly dmax (first point on the x axis)."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(extra, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = d * rng.uniform(1.0, 0.9 * dmax, size=(extra, 1))
    return np.concatenate([[[dmax, 0.0, 0.0]], pts], 0).astype(np.float32)


def tiny_map():
    rng = np.random.default_rng(0)
    return oracle.Map(rng.uniform(-5, 5, size=(200, 3)).astype(np.float32), 1.0, 6)


def test_city_grid_closed_form():
    """Eq. (2) and Sec. III-D evaluated by hand for r = 1 m, d_max = 100 m."""
    g = json.load(open(os.path.join(GOLDEN, "grid_city_dmax100.json")))
    m = tiny_map()
    rp = math.radians(3.0)
    lo = np.array([-250, -250, -0.2, -rp, -rp, 0.0], np.float32)
    hi = np.array([250, 250, 3.8, rp, rp, 2 * math.pi], np.float32)
    s = oracle.Search(m, one_point_scan(100.0), lo, hi)
    assert s.grid.dmax == pytest.approx(100.0, abs=1e-12)
    assert s.delta(0) == pytest.approx(g["delta0"], abs=5e-11)
    for l in range(7):
        # arccos(1 - x^2/2) = 2 asin(x/2): an independent closed form of Eq. (2)
        assert s.delta(l) == pytest.approx(2 * math.asin((2 ** l) / 200.0), rel=1e-10)
        assert s.n(2, l) == g["n_yaw"][l]
        assert s.n(0, l) == g["n_roll"][l] and s.n(1, l) == g["n_roll"][l]
        assert s.a(2, l) == g["a_yaw"][l]
        assert s.a(0, l) == g["a_roll"][l] and s.a(1, l) == g["a_roll"][l]
    assert s.lo == (-250, -250, 0) and s.hi == (250, 250, 3)


@pytest.mark.parametrize("seed", range(6))
def test_grid_invariants(seed):
    rng = np.random.default_rng(seed)
    r = float(rng.choice([0.25, 0.5, 1.0]))
    levels = int(rng.integers(0, 7))
    dmax = float(rng.uniform(5, 120))
    rp = float(rng.uniform(0.0, 0.2))
    lo = np.array([-10, -7.3, 0.4, -rp, -rp * 0.5, float(rng.uniform(-1, 0))], np.float32)
    hi = np.array([9.6, 7.7, 2.2, rp, rp, float(rng.uniform(0.5, 6.3))], np.float32)
    m = oracle.Map(rng.uniform(-5, 5, size=(100, 3)).astype(np.float32), r, levels)
    s = oracle.Search(m, one_point_scan(dmax, seed=seed), lo, hi)
    for ax in range(3):
        W = float(hi[3 + ax]) - float(lo[3 + ax])
        for l in range(levels + 1):
            n, dp, d = s.n(ax, l), s.dprime(ax, l), s.delta(l)
            if W == 0:
                assert n == 1
                continue
            assert n * dp == pytest.approx(W, rel=1e-12)       # equal segments cover W
            assert dp <= d * (1 + 1e-12)                        # each segment within delta(r_l)
            assert (n - 1) * d < W                              # and the fewest that do
            if l >= 1:
                a, n1 = s.a(ax, l), s.n(ax, l - 1)
                assert a == math.ceil(s.dprime(ax, l) / s.dprime(ax, l - 1) - 1e-9) if n1 > 1 else a == 1
                assert a * n >= n1 and (a - 1) * n < n1
                assert n <= n1
    for ax in range(3):
        assert s.lo[ax] == math.ceil(float(lo[ax]) / r)
        assert s.hi[ax] == math.floor(float(hi[ax]) / r)


def test_translation_only_grid():
    m = tiny_map()
    rp = math.radians(2.0)
    lo = np.array([-3, -3, 0, -rp, -rp, 0], np.float32)
    hi = np.array([3, 3, 1, rp, rp, 2 * math.pi], np.float32)
    s = oracle.Search(m, one_point_scan(30.0), lo, hi, translation_only=True)
    for ax in range(3):
        for l in range(7):
            assert s.n(ax, l) == s.n(ax, 0)
            assert s.a(ax, l) == 1 or l == 0


@pytest.mark.parametrize("angles", [(0.01, -0.02, 0.3), (0.0, 0.0, 3.0), (-0.05, 0.04, 5.9), (0.3, -0.2, 1.0)])
def test_rotation_convention(angles):
    """R = Rz(yaw) Ry(pitch) Rx(roll): scipy's extrinsic x-y-z Euler rotation."""
    roll, pitch, yaw = angles
    m = tiny_map()
    lo = np.array([0, 0, 0, roll, pitch, yaw], np.float32)
    s = oracle.Search(m, one_point_scan(10.0), lo, lo)
    R = s.rotation(0, 0, 0, 0)
    ref = Rotation.from_euler("xyz", [float(np.float32(a)) for a in angles]).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-7)


def expand_to_leaves(s, levels):
    """Apply the branching rule from every top-level node down to level 0."""
    top = []
    for x in range(s.lo[0] >> levels, (s.hi[0] >> levels) + 1):
        for y in range(s.lo[1] >> levels, (s.hi[1] >> levels) + 1):
            for z in range(s.lo[2] >> levels, (s.hi[2] >> levels) + 1):
                for a in range(s.n(0, levels)):
                    for b in range(s.n(1, levels)):
                        for c in range(s.n(2, levels)):
                            top.append((levels, x, y, z, a, b, c))
    frontier = top
    for _ in range(levels):
        nxt = []
        for nd in frontier:
            nxt.extend(tuple(int(v) for v in ch) for ch in s.children(nd))
        frontier = nxt
    return frontier


@pytest.mark.parametrize("translation_only", [False, True])
def test_every_leaf_reached_exactly_once(translation_only):
    """Branching from the top level reaches each leaf of the search set once."""
    rng = np.random.default_rng(1)
    m = oracle.Map(rng.uniform(-5, 5, size=(100, 3)).astype(np.float32), 0.5, 3)
    rp = math.radians(4.0)
    lo = np.array([-1.9, -1.2, 0.0, -rp, -rp, 0.0], np.float32)
    hi = np.array([1.6, 1.9, 0.7, rp, rp, 2 * math.pi], np.float32)
    s = oracle.Search(m, one_point_scan(4.0), lo, hi, translation_only=translation_only)
    leaves = expand_to_leaves(s, 3)
    cnt = Counter(leaves)
    assert max(cnt.values()) == 1
    want = {(0, x, y, z, a, b, c)
            for x in range(s.lo[0], s.hi[0] + 1) for y in range(s.lo[1], s.hi[1] + 1)
            for z in range(s.lo[2], s.hi[2] + 1) for a in range(s.n(0, 0))
            for b in range(s.n(1, 0)) for c in range(s.n(2, 0))}
    assert set(cnt) == want


def test_children_rule():
    """Children are (2c + j) in translation and (a c + j) in each angle, both
    kept only inside the search set, rotations outer and translations inner."""
    rng = np.random.default_rng(2)
    m = oracle.Map(rng.uniform(-5, 5, size=(100, 3)).astype(np.float32), 1.0, 6)
    rp = math.radians(3.0)
    lo = np.array([-250, -250, -0.2, -rp, -rp, 0.0], np.float32)
    hi = np.array([250, 250, 3.8, rp, rp, 2 * math.pi], np.float32)
    s = oracle.Search(m, one_point_scan(100.0), lo, hi)
    node = (4, 3, -2, 0, 0, 0, 39)   # yaw cell 39 of 40 at level 4: a = 2 -> 78, 79 (< 79 cells at l = 3)
    ch = s.children(node)
    a = [s.a(ax, 4) for ax in range(3)]
    exp = []
    for ja in range(a[0]):
        for jb in range(a[1]):
            for jg in range(a[2]):
                ang = (a[0] * 0 + ja, a[1] * 0 + jb, a[2] * 39 + jg)
                if any(ang[i] >= s.n(i, 3) for i in range(3)):
                    continue
                for jx in (0, 1):
                    for jy in (0, 1):
                        for jz in (0, 1):
                            t = (6 + jx, -4 + jy, 0 + jz)
                            if not all((s.lo[i] >> 3) <= t[i] <= (s.hi[i] >> 3) for i in range(3)):
                                continue
                            exp.append((3,) + t + ang)
    assert [tuple(int(v) for v in c) for c in ch] == exp
    assert len(exp) == 2 * 2 * 1 * 4 * 1   # z: only cell 0 at level 3; roll, pitch 2 each; yaw 78 only
