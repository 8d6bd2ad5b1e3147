"""Full-size parity on the city workload: every query the benchmark times.

The expected results are the CPU oracle's, stored in
`tests/golden/city_localize.json` by `tests/golden/make_city_golden.py` (which
calls only `oracle/` and the seeded generators).  Each query is regenerated
here and its scan is checked against the stored sha256 first, so a drift of
the generator cannot pass as a parity failure or a pass.

Every result field is compared bit-exactly (found, score, leaf, pose as
float32, nodes expanded / scored, flushes, leaves accepted, initial set) for
the per-iteration launches, the persistent kernel and the graph-captured
iterations.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import paper_2310_10023_amd as bbs
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "city_localize.json")
FIELDS = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
          "initial_size", "initial_kept")
MODES = {"launches": {}, "persistent": {"persistent": True}, "graph": {"graph": True}}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load_golden():
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        return json.load(f)


DOC = load_golden()


def cases():
    if DOC is None:
        return []
    out = []
    for name, c in DOC["cases"].items():
        for seed in sorted(c["queries"], key=int):
            out.append((name, int(seed)))
    return out


@pytest.fixture(scope="module")
def city_map():
    import torch
    c = synth.city_scene(1000)
    assert hashlib.sha256(np.ascontiguousarray(c.points).tobytes()).hexdigest() == DOC["map"]["points_sha256"]
    say("city map points", len(c.points))
    return c, bbs.Map(torch.from_numpy(c.points).cuda(), DOC["map"]["r"], DOC["map"]["levels"]), bbs.Workspace()


def check(got, want, label):
    for key in FIELDS:
        assert got[key] == want[key], (label, key, got[key], want[key])
    if want["found"]:
        np.testing.assert_array_equal(np.float32(got["pose"]), np.float32(want["pose"]), err_msg=label)


@pytest.mark.skipif(DOC is None, reason="tests/golden/city_localize.json has not been written")
@pytest.mark.parametrize("case,seed", cases())
def test_city_query_equals_stored_oracle(city_map, case, seed):
    import torch
    c, gmap, ws = city_map
    spec = DOC["cases"][case]
    want = spec["queries"][str(seed)]
    scan = synth.city_query(c, seed, spec["k"], voxel=spec["voxel"])
    assert hashlib.sha256(np.ascontiguousarray(scan.points).tobytes()).hexdigest() == want["scan_sha256"]
    lo = np.array(DOC["range"]["min"], np.float32)
    hi = np.array(DOC["range"]["max"], np.float32)
    dev = torch.from_numpy(scan.points).cuda()
    for mode, kw in MODES.items():
        say(f"city {case} seed {seed} {mode}: k {spec['k']} b {spec['batch']} "
            f"(oracle scored {want['nodes_scored']})")
        got = bbs.localize(gmap, dev, lo, hi, spec["threshold"], batch_size=spec["batch"], workspace=ws,
                           nested_angles=bool(spec.get("nested", False)), **kw)
        check(got, want, f"{case}/{seed}/{mode}")
        if mode == "persistent":
            assert got["persistent_used"] == 1


@pytest.mark.skipif(DOC is None, reason="tests/golden/city_localize.json has not been written")
def test_city_stream_equals_stored_oracle(city_map):
    """Stream serving on the city (concurrent workers, each with its own
    workspace and stream, Poisson arrivals) gives the stored oracle result
    of every query, including one that exhausts the tree."""
    c, gmap, _ = city_map
    spec = DOC["cases"]["bench"]
    seeds = [14, 16, 17, 15, 8, 0, 13, 10, 3, 2]
    scans = []
    for s in seeds:
        sc = synth.city_query(c, s, spec["k"], voxel=spec["voxel"])
        assert hashlib.sha256(np.ascontiguousarray(sc.points).tobytes()).hexdigest() == \
            spec["queries"][str(s)]["scan_sha256"]
        scans.append(sc.points)
    lo = np.array(DOC["range"]["min"], np.float32)
    hi = np.array(DOC["range"]["max"], np.float32)
    arrivals = np.cumsum(np.random.default_rng(1).exponential(0.003, size=len(seeds)))
    say("city stream", len(seeds), "queries, 4 workers")
    res, t0, t1 = bbs.serve(gmap, scans, [(lo, hi)] * len(seeds), [spec["threshold"]] * len(seeds), arrivals,
                            workers=4, batch_size=spec["batch"])
    for s, got in zip(seeds, res):
        check(got, spec["queries"][str(s)], f"stream/{s}")
    assert np.all(t1 >= t0) and np.all(t0 >= arrivals - 1e-6)
