"""Pins for the oracle's search schedule (Alg. 2, Sec. III-E).

The paper prints no node counts, so the schedule is pinned by hand: two tiny
instances (`tests/golden/schedule_hand.json`) whose node scores can be read
off the voxel sets by eye, with every pop, flush, counter and the match
traced by hand from the rules of Alg. 2 and the readings the oracle states
(queue order score desc, level asc, first in first out; strict `<` prune;
flush when more than b children are pending, and when the queue runs empty),
each also traced in the depth-first order of Alg. 1 (level asc, then score
desc, then first in first out).

The mutation tests show that these pins bind: each of seven plausible slips in
the schedule (level order reversed, last in first out, flush at >= b, no
termination flush, prune at <=, and in the depth-first order levels reversed
or the best-first order used instead) is planted in a copy of the oracle's source,
compiled, and must fail the hand-traced pins (run in a subprocess that loads
the broken copy); the unmodified copy must pass them.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "schedule_hand.json")
with open(GOLDEN) as _f:
    INSTANCES = json.load(_f)["instances"]


def build_instance(inst):
    """Map points at voxel centres, scan points at key centres, r = 1, every
    angular range fixed at 0 and y, z fixed to leaf cell 0."""
    vox = np.array(inst["map_voxels_x"], np.float64)
    pts = np.stack([vox + 0.5, np.full(len(vox), 0.5), np.full(len(vox), 0.5)], 1).astype(np.float32)
    keys = np.array(inst["scan_keys_x"], np.float64)
    scan = np.stack([keys + 0.5, np.full(len(keys), 0.5), np.full(len(keys), 0.5)], 1).astype(np.float32)
    x0, x1 = inst["x_range"]
    lo = np.array([x0, 0, 0, 0, 0, 0], np.float32)
    hi = np.array([x1, 0, 0, 0, 0, 0], np.float32)
    m = oracle.Map(pts, 1.0, inst["levels"])
    return m, oracle.Search(m, scan, lo, hi)


@pytest.mark.parametrize("inst", INSTANCES, ids=[i["name"] for i in INSTANCES])
def test_hand_traced_voxel_sets_and_scores(inst):
    m, s = build_instance(inst)
    for l in range(inst["levels"] + 1):
        want = {(x, y, z) for x in inst["D_x"][str(l)] for y in (-1, 0) for z in (-1, 0)}
        assert {tuple(v) for v in m.level_keys(l).tolist()} == want, l
        for c, sc in inst["scores"][str(l)].items():
            assert s.score(l, int(c), 0, 0, 0, 0, 0) == sc, (l, c)
    # the rotation is exactly the identity
    np.testing.assert_array_equal(s.rotation(0, 0, 0, 0), np.eye(3, dtype=np.float32))


@pytest.mark.parametrize("inst", INSTANCES, ids=[i["name"] for i in INSTANCES])
def test_hand_traced_schedule(inst):
    _, s = build_instance(inst)
    r = s.localize(inst["threshold"], batch=inst["batch"], threads=1, trace_cap=64, events_cap=64,
                   strategy=inst.get("strategy", "best_first"))
    assert r["events"] == inst["events"]
    want = inst["result"]
    got = {k: r[k] for k in want if k != "flush_sizes"}
    got["flush_sizes"] = r["flush_sizes"]
    assert got == want


MUTANTS = {
    "level_order_reversed": ("if (a->level != b->level) return a->level < b->level;",
                             "if (a->level != b->level) return a->level > b->level;"),
    "last_in_first_out": ("return a->seq < b->seq;", "return a->seq > b->seq;"),
    "flush_at_b": ("if (pending.n > batch) flush = 1;", "if (pending.n >= batch) flush = 1;"),
    "no_termination_flush": ("if (pending.n == 0) break;\n            flush = 1;",
                             "break;\n            flush = 1;"),
    "prune_at_equal": ("if (c.score < best) {", "if (c.score <= best) {"),
    "depth_first_levels_reversed": ("if (order == ORC_DEPTH_FIRST && a->level != b->level) return a->level < b->level;",
                                    "if (order == ORC_DEPTH_FIRST && a->level != b->level) return a->level > b->level;"),
    "depth_first_as_best_first": ("if (order == ORC_DEPTH_FIRST && a->level != b->level)",
                                  "if (order == 99 && a->level != b->level)"),
}


def _run_pins_with(lib_path):
    env = dict(os.environ, BBS_ORACLE_LIB=lib_path)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", os.path.abspath(__file__),
           "-k", "hand_traced"]
    return subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=300)


@pytest.mark.parametrize("name", [None] + list(MUTANTS), ids=["unmodified"] + list(MUTANTS))
def test_pins_kill_schedule_mutants(name, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "bbs_oracle.c")).read()
    if name is not None:
        old, new = MUTANTS[name]
        assert src.count(old) == 1, name
        src = src.replace(old, new)
    path = tmp_path / "mut.c"
    path.write_text(src)
    lib_path = oracle.compile_source(str(path), str(tmp_path / "libmut.so"))
    res = _run_pins_with(lib_path)
    if name is None:
        assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    else:
        assert res.returncode == 1 and "failed" in res.stdout, res.stdout[-2000:] + res.stderr[-2000:]
