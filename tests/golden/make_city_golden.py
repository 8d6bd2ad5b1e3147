#!/usr/bin/env python3
"""Write the oracle's full localization results on the city workload.

The stored file is what the GPU parity tests and the benchmark compare the HIP
library against at full size.  It is written by the CPU oracle only (this
script imports nothing but `oracle` and the seeded input generators in
`synth`); no value in it comes from the GPU path.

Workload: city seed 1000 (500 x 500 x 30 m, about 10.4M points), r = 1 m,
l_max = 6, search x, y +-250 m, z 1.8 +- 2 m, roll/pitch +-3 deg, yaw
[0, 2 pi), threshold = ceil(0.95 K).  Cases:
  bench    K = 10,000 (0.5 m thinning), b = 10,000, query seeds 0..19 -- the
           queries the benchmark times;
  tuned    b = 64,000 at K = 5,000 / 10,000 / 20,000 (0.25 m thinning), query
           seeds 0 and 1 -- the batch size the autotuner picks;
  nested   as bench, on the nested angular grid (option nested_angles).
Each query records every result field, the sha256 of its scan (so a reader
can check it regenerated the same input), and the oracle's wall time and
thread count on the machine that wrote it.

    python tests/golden/make_city_golden.py [--threads 7] [--only bench]

The script is resumable: queries already in the file are kept.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "city_localize.json")
MAP_SEED = 1000
R, LEVELS = 1.0, 6
CASES = {
    "bench": {"k": 10000, "voxel": 0.5, "batch": 10000, "seeds": list(range(20))},
    "tuned_k5000": {"k": 5000, "voxel": 0.25, "batch": 64000, "seeds": [0, 1]},
    "tuned_k10000": {"k": 10000, "voxel": 0.25, "batch": 64000, "seeds": [0, 1]},
    "tuned_k20000": {"k": 20000, "voxel": 0.25, "batch": 64000, "seeds": [0, 1]},
    "nested": {"k": 10000, "voxel": 0.5, "batch": 10000, "seeds": list(range(20)), "nested": True},
}
FIELDS = ("found", "score", "leaf", "pose", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
          "initial_size", "initial_kept", "bound_checks", "bound_violations")


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def save(doc):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--only", default=None, help="comma-separated case names")
    args = ap.parse_args()
    city = synth.city_scene(MAP_SEED)
    lo, hi = synth.search_range_city()
    doc = {"map": {"scene": f"synth.city_scene({MAP_SEED})", "points": int(len(city.points)),
                   "points_sha256": sha(city.points), "r": R, "levels": LEVELS},
           "range": {"min": [float(v) for v in lo], "max": [float(v) for v in hi]},
           "cases": {}}
    if os.path.exists(OUT):
        with open(OUT) as f:
            old = json.load(f)
        if old.get("map") == doc["map"] and old.get("range") == doc["range"]:
            doc["cases"] = old.get("cases", {})
    omap = oracle.Map(city.points, R, LEVELS)
    names = args.only.split(",") if args.only else list(CASES)
    for name in names:
        c = CASES[name]
        T = synth.threshold_95(c["k"])
        case = doc["cases"].setdefault(name, {})
        case.update({"k": c["k"], "voxel": c["voxel"], "batch": c["batch"], "threshold": T,
                     "scan": f"synth.city_query(city, seed, {c['k']}, voxel={c['voxel']})"})
        if c.get("nested"):
            case["nested"] = True
        queries = case.setdefault("queries", {})
        for seed in c["seeds"]:
            if str(seed) in queries:
                continue
            scan = synth.city_query(city, seed, c["k"], voxel=c["voxel"])
            s = oracle.Search(omap, scan.points, lo, hi, nested=bool(c.get("nested")))
            t0 = time.perf_counter()
            r = s.localize(T, batch=c["batch"], threads=args.threads)
            dt = time.perf_counter() - t0
            q = {f: r[f] for f in FIELDS}
            q.update({"scan_sha256": sha(scan.points), "true_pose": [float(v) for v in scan.pose],
                      "oracle_s": round(dt, 2), "oracle_threads": args.threads})
            queries[str(seed)] = q
            save(doc)
            print(f"{name} seed {seed}: found {r['found']} score {r['score']} scored {r['nodes_scored']} "
                  f"expanded {r['nodes_expanded']} in {dt:.0f} s", flush=True)
    save(doc)


if __name__ == "__main__":
    main()
