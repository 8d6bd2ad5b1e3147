"""Pins of the nested angular grid (an alternative reading of Eqs. (13)-(15),
`orc_grid_nest`): every cell splits into exactly a equal children, each level
keeps steps at most delta(r_l), the top level is Eq. (13)'s, and the search
on it is exact where the bound is (translation-only, and the exact rotational
bound), and it shows the drift it removes."""
import math

import numpy as np
import pytest

import oracle
import synth


def searches(seed=0, k=150, rp_deg=2.0, yaw=2 * math.pi):
    scene = synth.tiny_scene(seed, n_map=500)
    scan = synth.scan_scene(scene, seed, k, z=1.0, rp_deg=rp_deg, n_beams=16, n_az=256, max_range=12.0).points
    rp = math.radians(rp_deg)
    lo = np.array([-2, -2, 0.5, -rp, -rp, 0.0], np.float32)
    hi = np.array([2, 2, 1.5, rp, rp, yaw], np.float32)
    m = oracle.Map(scene.points, 0.5, 3)
    return (oracle.Search(m, scan, lo, hi), oracle.Search(m, scan, lo, hi, nested=True), scene, scan, lo, hi)


def test_cells_nest_exactly_and_stay_below_delta():
    city = synth.city_scene(1000)
    lo, hi = synth.search_range_city()
    m = oracle.Map(city.points[:500], 1.0, 6)
    for seed in range(6):
        sc = synth.city_query(city, seed, 10000, voxel=0.5)
        p = oracle.Search(m, sc.points, lo, hi)
        s = oracle.Search(m, sc.points, lo, hi, nested=True)
        for ax in range(3):
            W = float(hi[3 + ax]) - float(lo[3 + ax])
            assert s.n(ax, 6) == p.n(ax, 6) == math.ceil(W / s.delta(6) - 1e-12) or W == 0
            for l in range(1, 7):
                a = s.a(ax, l)
                assert s.n(ax, l - 1) == a * s.n(ax, l)
                # cell c of level l spans exactly its children a c .. a c + a - 1
                assert abs(a * s.dprime(ax, l - 1) - s.dprime(ax, l)) < 1e-12 * max(W, 1)
            for l in range(0, 7):
                if W > 0:
                    assert s.dprime(ax, l) <= s.delta(l) + 1e-15


def test_literal_grid_drifts_where_ratios_are_not_integers():
    """City query 2 (the grid of the literal reading there: 629, 315, 157, ...
    yaw cells) has a = 3 at level 2: its cell 100 centres at 4.02 rad, its
    children at about 6.01 rad (1.5 times).  The nested grid keeps them
    inside their parent."""
    city = synth.city_scene(1000)
    lo, hi = synth.search_range_city()
    m = oracle.Map(city.points[:500], 1.0, 6)
    sc = synth.city_query(city, 2, 10000, voxel=0.5)
    p = oracle.Search(m, sc.points, lo, hi)
    assert p.a(2, 2) == 3
    centre = lambda s, c, l: float(lo[5]) + s.dprime(2, l) * (c + 0.5)
    kids = [centre(p, 3 * 100 + j, 1) for j in range(3)]
    assert abs(np.mean(kids) - 1.5 * centre(p, 100, 2)) < 0.05
    s = oracle.Search(m, sc.points, lo, hi, nested=True)
    a = s.a(2, 2)
    for c in (0, 100, s.n(2, 2) - 1):
        kids = [centre(s, a * c + j, 1) for j in range(a)]
        lo_c, hi_c = centre(s, c, 2) - s.dprime(2, 2) / 2, centre(s, c, 2) + s.dprime(2, 2) / 2
        assert all(lo_c < x < hi_c for x in kids)


@pytest.mark.parametrize("seed", [0, 2])
def test_nested_translation_only_equals_literal(seed):
    scene = synth.tiny_scene(seed, n_map=500)
    scan = synth.scan_scene(scene, seed, 120, z=1.0, rp_deg=1.0, n_beams=16, n_az=256, max_range=12.0).points
    lo = np.array([-2, -2, 0.5, -0.02, -0.02, 0.0], np.float32)
    hi = np.array([2, 2, 1.5, 0.02, 0.02, 1.0], np.float32)
    m = oracle.Map(scene.points, 0.5, 3)
    a = oracle.Search(m, scan, lo, hi, translation_only=True).localize(60, batch=64, threads=8)
    b = oracle.Search(m, scan, lo, hi, translation_only=True, nested=True).localize(60, batch=64, threads=8)
    assert a == b


@pytest.mark.parametrize("seed,frac", [(0, 0.5), (1, 0.8)])
def test_nested_exact_bound_search_equals_full_search(seed, frac):
    scene = synth.tiny_scene(seed, n_map=500)
    scan = synth.scan_scene(scene, seed, 120, z=1.0, rp_deg=1.0, n_beams=16, n_az=256, max_range=12.0).points
    rp = math.radians(1.0)
    lo = np.array([-2, -2, 0.5, -rp, -rp, 0.0], np.float32)
    hi = np.array([2, 2, 1.5, rp, rp, 1.2], np.float32)
    need = oracle.Search(oracle.Map(scene.points, 0.5, 3), scan, lo, hi, nested=True).margins_needed()
    s = oracle.Search(oracle.Map(scene.points, 0.5, 3, margins=need), scan, lo, hi, rot_exact=True, nested=True)
    sc = s.all_leaf_scores(threads=8)
    T = int(math.ceil(frac * len(scan)))
    i = int(np.argmax(sc.ravel()))
    idx = np.unravel_index(i, sc.shape)
    want = (int(sc.ravel()[i]), [int(idx[0]) + s.lo[0], int(idx[1]) + s.lo[1], int(idx[2]) + s.lo[2],
                                 int(idx[3]), int(idx[4]), int(idx[5])])
    for b in (1, 64, 10000):
        r = s.localize(T, batch=b, threads=8)
        if want[0] < T:
            assert r["found"] == 0
        else:
            assert (r["score"], r["leaf"]) == want, b
