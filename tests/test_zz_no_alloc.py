"""bbs_localize_noalloc (no device allocation, static per-GPU scratch) gives
the results of bbs_localize, call after call on the shared scratch."""
import sys

import numpy as np
import pytest

import paper_2310_10023_amd as bbs
import synth

pytestmark = pytest.mark.gpu

FIELDS = ("found", "score", "leaf", "pose", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
          "initial_size", "initial_kept", "seeded", "seed_score")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b, label):
    for f in FIELDS:
        assert a[f] == b[f], (label, f, a[f], b[f])


def test_noalloc_equals_localize_on_consecutive_calls():
    import torch
    scene = synth.room_scene(0)
    gmap = bbs.Map(scene.points, 0.5, 4)
    lo, hi = synth.search_range_room()
    ws = bbs.Workspace()
    # the second call is smaller (fewer points, smaller batch), so it runs on
    # whatever the first left in the scratch
    calls = [(3, 2000, 10000, {}), (5, 1500, 700, {}), (1, 1200, 64, {"persistent": True})]
    prior = np.random.default_rng(4).normal(size=1088).astype(np.float32)
    calls.append((2, 1000, 2000, {"prior": prior, "seed_beam": 8}))
    for seed, k, b, kw in calls:
        sc = synth.room_query(scene, seed, k)
        T = synth.threshold_95(k)
        say("noalloc room seed", seed, "k", k, "b", b, sorted(kw))
        want = bbs.localize(gmap, sc.points, lo, hi, T, batch_size=b, workspace=ws, **kw)
        got = bbs.localize_noalloc(gmap, torch.from_numpy(sc.points).cuda(), lo, hi, T, batch_size=b, **kw)
        same(got, want, (seed, k, b))
        got2 = bbs.localize_noalloc(gmap, sc.points, lo, hi, T, batch_size=b, **kw)   # host scan
        same(got2, want, (seed, k, b, "host"))
        assert got["found"] == 1


def test_noalloc_rejects_allocating_options_and_oversized_searches():
    scene = synth.room_scene(0)
    gmap = bbs.Map(scene.points, 0.5, 4)
    lo, hi = synth.search_range_room()
    sc = synth.room_query(scene, 3, 500)
    opt = bbs.Options()
    L = bbs.lib()
    L.bbs_default_options(opt)
    opt.profile = 1
    rng = bbs._range(lo, hi)
    res = bbs.Result()
    import ctypes as C
    assert L.bbs_localize_noalloc(gmap.handle, sc.points.ctypes.data, len(sc.points), 0, C.byref(rng), 400,
                                  C.byref(opt), C.byref(res)) == -1
    assert b"profile and graph" in L.bbs_last_error()
    # a batch whose tile tables alone exceed the scratch: clear error, nothing runs
    with pytest.raises(bbs.BbsError) as e:
        bbs.localize_noalloc(gmap, sc.points, lo, hi, 0, batch_size=1 << 24)
    assert e.value.status == -1
    # and the scratch still serves a normal call afterwards
    r = bbs.localize_noalloc(gmap, sc.points, lo, hi, synth.threshold_95(500), batch_size=1000)
    assert r["found"] == 1
