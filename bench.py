#!/usr/bin/env python3
"""Benchmark of 3D-BBS global localization on one AMD Instinct MI355X.

Workload: the outdoor city (seeded procedural 500 x 500 x 30 m block grid,
about 10.4M map points), voxel map r = 1.0 m with l_max = 6, 10,000-point
ray-cast scans, search x, y +-250 m, z +-2 m, roll/pitch +-3 deg, yaw 360 deg,
score threshold 95 % of the scan, plain batched branch and bound with
b = 10,000.  One step = one localization of one scan (the whole hot path:
scan set-up, initial set, and the gather / branch / score / push loop until
the queue is exhausted).  The map and every scan are resident in GPU memory
before the timed region starts.

Prints one JSON line (value = nodes scored per second over the timed steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "nodes scored/s and ms per localization, plain vs learned-order BnB, 1 GPU"
HBM_PEAK_GBS = 8000.0
# 32-bit VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (the 157.3 TFLOP/s fp32 vector figure counts a packed FMA as 4 flops per lane-op)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# A model of the ALU work per (node, scan point), kept for reference only: 15 fp32
# ops of the 3x3 transform and 3 floors shared by the 8 translational siblings of
# a rotation, plus about 10 integer ops
MODEL_OPS_PER_NODE_POINT = 18 / 8 + 10
# Algorithmic bytes of one lookup of the brick-column layout: the 8-byte column
# entry answers a whole group of translational siblings for one scan point, and
# the 12-byte scan point is read for it
ALG_BYTES_PER_LOOKUP = 8 + 12
# The timed localizations bracket every PROFILE_EVERY-th scoring launch with a
# pair of HIP events on the library's stream; the mean of those launches gives
# the kernel's duration.  Bracketing every launch added about 9 % to the
# localization time (each event pair adds queue time between the kernels).
PROFILE_EVERY = 8
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_score_city_traffic.md")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_score_city_counters.md")
GOLDEN_FILE = os.path.join(ROOT, "tests", "golden", "city_localize.json")
WEIGHTS = os.path.join(ROOT, "paper_2310_10023_amd", "proposal_weights.npz")
SCORE_SRC = os.path.join(ROOT, "paper_2310_10023_amd", "csrc", "bbs_search.hip")


def score_kernel_sha() -> str:
    """Hash of the scoring kernel's source (its section of the search source)."""
    text = open(SCORE_SRC).read()
    m = re.search(r"// -+ scoring \(Eq\. \(12\), Sec\. III-C\)\n.*?// -+ initial set", text, flags=re.S)
    return hashlib.sha256((m.group(0) if m else text).encode()).hexdigest()[:16]


def profile_record(path):
    """The machine-readable record of a committed profile summary, or None
    when it is missing or was taken on other scoring-kernel code."""
    try:
        text = open(path).read()
        m = re.search(r"```json\n(.*?)\n```", text, flags=re.S)
        d = json.loads(m.group(1)) if m else {}
    except (OSError, ValueError):
        return None
    return d if d.get("kernel_sha") == score_kernel_sha() else None


def rot_error(a, b):
    """Angle (rad) of the relative rotation between two roll/pitch/yaw triples."""
    import math

    import numpy as np

    import synth
    Ra, Rb = synth.rotation_zyx(*a), synth.rotation_zyx(*b)
    return math.acos(max(-1.0, min(1.0, (float(np.trace(Ra.T @ Rb)) - 1.0) / 2.0)))


def success(result, true_pose):
    """The success criterion of Sec. IV: translation error below 2.0 m and
    rotation error below 0.05 rad."""
    import numpy as np
    if not result["found"]:
        return False
    p = np.array(result["pose"], np.float64)
    return float(np.linalg.norm(p[:3] - true_pose[:3])) < 2.0 and rot_error(p[3:], true_pose[3:]) < 0.05


def pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(q * len(v)))] if v else None


def golden_parity(results, seeds, k, batch, case_name="bench"):
    """How many timed results equal the oracle's stored results (every field)."""
    try:
        doc = json.load(open(GOLDEN_FILE))
    except (OSError, ValueError):
        return None
    case = doc.get("cases", {}).get(case_name, {})
    if case.get("k") != k or case.get("batch") != batch:
        return None
    q = case.get("queries", {})
    keys = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes", "leaves_accepted",
            "initial_size", "initial_kept")
    n = eq = 0
    for s, r in zip(seeds, results):
        w = q.get(str(s))
        if w is None:
            continue
        n += 1
        eq += all(r[f] == w[f] for f in keys)
    return (f"{eq}/{n} equal to {os.path.relpath(GOLDEN_FILE, ROOT)} case {case_name} (of {len(seeds)} timed queries)"
            if n else None)


def with_one_core(fn):
    """Run fn() with this thread pinned to one host core; returns (result, core)."""
    old = os.sched_getaffinity(0)
    core = max(old)
    os.sched_setaffinity(0, {core})
    try:
        return fn(), core
    finally:
        os.sched_setaffinity(0, old)


def cpu_baseline(points, scan, lo, hi, T, batch, seconds):
    """The oracle (unchanged) on the same workload, bounded to a few seconds
    of CPU work each: the first nodes of the first timed query's search, on
    one pinned core (single thread) and with OpenMP over each scored batch."""
    import oracle
    omap = oracle.Map(points, 1.0, 6)
    s = oracle.Search(omap, scan, lo, hi)

    def sample(threads, secs):
        t0 = time.perf_counter()
        probe = s.localize(T, batch=batch, threads=threads, max_scored=1000)
        rate = probe["nodes_scored"] / max(time.perf_counter() - t0, 1e-6)
        budget = int(max(1000, rate * secs))
        t0 = time.perf_counter()
        r = s.localize(T, batch=batch, threads=threads, max_scored=budget)
        dt = time.perf_counter() - t0
        return r["nodes_scored"], dt

    (n1, dt1), core = with_one_core(lambda: sample(1, seconds / 2))
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    nm, dtm = sample(threads, seconds / 2)
    return {"value": n1 / dt1, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n1} nodes scored of the search of query seed 0, single thread pinned to host core "
                      f"{core}, {dt1:.1f} s",
            "multi_thread": {"value": nm / dtm, "unit": "nodes/s", "cores": threads,
                             "sample": f"first {nm} nodes scored of the same search, OpenMP over each scored batch, "
                                       f"{dtm:.1f} s"}}


def indoor_leg(seconds):
    """The tiny indoor configuration: room 20 x 20 x 5 m, r = 0.5 m, l_max = 4,
    2,000-point scans, plain BnB at b = 10,000.  GPU ms per localization over
    query seeds 0..19, and the oracle's CPU seconds per localization (single
    thread, one pinned core) on as many of the same seeds as fit in `seconds`."""
    import numpy as np
    import torch

    import oracle
    import paper_2310_10023_amd as bbs
    import synth
    scene = synth.room_scene(0)
    lo, hi = synth.search_range_room()
    T = synth.threshold_95(2000)
    scans = [synth.room_query(scene, s, 2000) for s in range(20)]
    gmap = bbs.Map(torch.from_numpy(scene.points).cuda(), 0.5, 4)
    dev = [torch.from_numpy(sc.points).cuda() for sc in scans]
    ws = bbs.Workspace()
    bbs.localize(gmap, dev[0], lo, hi, T, workspace=ws)
    gpu_ms, res = [], []
    for d in dev:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res.append(bbs.localize(gmap, d, lo, hi, T, workspace=ws))
        torch.cuda.synchronize()
        gpu_ms.append((time.perf_counter() - t0) * 1e3)
    omap = oracle.Map(scene.points, 0.5, 4)

    def run_oracle():
        out = []
        t_end = time.perf_counter() + seconds
        for sc, g in zip(scans, res):
            if time.perf_counter() > t_end:
                break
            t0 = time.perf_counter()
            w = oracle.Search(omap, sc.points, lo, hi).localize(T, batch=10000, threads=1)
            out.append(((time.perf_counter() - t0) * 1e3, w, g))
        return out

    runs, core = with_one_core(run_oracle)
    keys = ("found", "score", "leaf", "nodes_expanded", "nodes_scored", "flushes")
    cpu_ms = [m for m, _, _ in runs]
    return {
        "workload": f"room 20x20x5 m seed 0 ({len(scene.points)} pts), r=0.5 m, l_max=4, 2000-pt scans (query seeds "
                    "0..19), roll/pitch +-2 deg, threshold 1900, b=10000, plain batched BnB",
        "gpu_ms_per_localization_p50": pct(gpu_ms, 0.5), "gpu_ms_per_localization_p99": pct(gpu_ms, 0.99),
        "gpu_ms_per_localization_mean": float(np.mean(gpu_ms)),
        "found": f"{sum(r['found'] for r in res)}/{len(res)}",
        "success_2m_0p05rad": f"{sum(success(r, sc.pose) for r, sc in zip(res, scans))}/{len(res)}",
        "oracle_cpu_s_per_localization_p50": pct(cpu_ms, 0.5) / 1e3 if cpu_ms else None,
        "oracle_cpu_s_per_localization_p99": pct(cpu_ms, 0.99) / 1e3 if cpu_ms else None,
        "oracle_queries": len(runs), "oracle_cores": 1, "oracle_core": core,
        "oracle_equal_to_gpu": f"{sum(all(w[f] == g[f] for f in keys) for _, w, g in runs)}/{len(runs)}",
    }


def timed_leg(gmap, dev, seeds, lo, hi, T, batch, ws, **kw):
    import torch

    import paper_2310_10023_amd as bbs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [bbs.localize(gmap, dev[s], lo, hi, T, batch_size=batch, workspace=ws, **kw) for s in seeds]
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=10000, help="scan points")
    ap.add_argument("--batch", type=int, default=10000, help="b")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU seconds of each bounded oracle sample (city: split over 1 core and all cores; indoor)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--details", default=None, help="write per-step results to this JSON file")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (to scale HBM byte counters) and exit")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-order comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="time the plain launches only (no persistent, graph, indoor or bandwidth legs)")
    ap.add_argument("--beam", type=int, default=8, help="seed beam width of the learned-order search")
    ap.add_argument("--stream", action="store_true",
                    help="run the 256-query stream workload instead (throughput, p50/p99 latency)")
    ap.add_argument("--stream-queries", type=int, default=256)
    ap.add_argument("--stream-workers", type=int, default=4)
    ap.add_argument("--tuned", action="store_true",
                    help="run the autotuned workload instead: scans of 5k/10k/20k points; batch size, scoring tile "
                         "and loop form (launches or persistent kernel) autotuned per scan size on separate "
                         "sample queries")
    ap.add_argument("--tuned-queries", type=int, default=20)
    ap.add_argument("--table1", action="store_true",
                    help="run the nine configurations of the paper's Table I (processing type x branching x search "
                         "strategy) on the tiny indoor workload instead")
    ap.add_argument("--table1-k", type=int, default=1000, help="scan points of the Table I workload")
    ap.add_argument("--table1-queries", type=int, default=10)
    ap.add_argument("--rot-exact", action="store_true",
                    help="the city queries with the exact rotational bound against plain (grown map tables)")
    ap.add_argument("--nested", action="store_true", help="with --rot-exact: on the nested angular grid")
    ap.add_argument("--net", action="store_true",
                    help="the proposal network instead: training step, inference and device prior (MFMA kernels)")
    ap.add_argument("--net-batch", type=int, default=128, help="training batch of --net")
    ap.add_argument("--table1-cpu-seconds", type=float, default=20.0,
                    help="CPU seconds each CPU configuration of Table I may spend (it runs as many queries as fit)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not an implemented path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2310_10023_amd as bbs
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.arange(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "copies": 5}))
        return
    if args.stream:
        return stream_bench(args)
    if args.tuned:
        return tuned_bench(args)
    if args.table1:
        return table1_bench(args)
    if args.rot_exact:
        return rot_exact_bench(args)
    if args.net:
        return net_bench(args)
    t0 = time.perf_counter()
    city = synth.city_scene(1000)
    lo, hi = synth.search_range_city()
    T = synth.threshold_95(args.k)
    warm_seeds = list(range(100, 100 + args.warmup))
    seeds = list(range(args.steps))
    scans = {s: synth.city_query(city, s, args.k, voxel=0.5) for s in warm_seeds + seeds}
    print(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s: {len(city.points)} map points, "
          f"{len(scans)} scans of {args.k}", file=sys.stderr, flush=True)

    pts = torch.from_numpy(city.points).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gmap = bbs.Map(pts, 1.0, 6)
    torch.cuda.synchronize()
    map_ms = (time.perf_counter() - t0) * 1e3
    dev = {s: torch.from_numpy(v.points).cuda() for s, v in scans.items()}
    ws = bbs.Workspace()
    for s in warm_seeds:
        bbs.localize(gmap, dev[s], lo, hi, T, batch_size=args.batch, profile=PROFILE_EVERY, workspace=ws)
    torch.cuda.synchronize()

    results, elapsed = timed_leg(gmap, dev, seeds, lo, hi, T, args.batch, ws, profile=PROFILE_EVERY)
    print(f"[bench] timed {len(seeds)} localizations in {elapsed:.3f} s", file=sys.stderr, flush=True)

    nodes = sum(r["nodes_scored"] for r in results)
    groups = sum(r["score_groups"] for r in results)
    launches = sum(r["score_launches"] for r in results)
    kern_ms = sum(r["score_kernel_ms"] for r in results)
    t_launch = kern_ms / max(launches, 1) * 1e-3            # seconds per scoring launch
    lookups = groups * args.k / max(launches, 1)              # group lookups per launch
    lat = [r["phase_ms"][3] for r in results]
    found_ms = [m for m, r in zip(lat, results) if r["found"]]
    lost_ms = [m for m, r in zip(lat, results) if not r["found"]]
    ok = sum(success(r, scans[s].pose) for s, r in zip(seeds, results))

    cnt = profile_record(COUNTERS_FILE)
    traffic = profile_record(TRAFFIC_FILE)
    valu_per_lookup = cnt.get("valu_lane_instr_per_lookup") if cnt else None
    achieved = valu_per_lookup * lookups / t_launch / 1e12 if valu_per_lookup and t_launch > 0 else None
    roofline = {
        "bound": "alu",
        "achieved": achieved,
        "peak": VALU_PEAK_TOPS,
        "unit": "T VALU lane-instructions/s (issued: SQ_INSTS_VALU x 64 per lookup from the counter profile x live "
                "lookups per launch / live launch time)",
        "frac": achieved / VALU_PEAK_TOPS if achieved else None,
        "traffic": traffic.get("bytes_per_launch") if traffic else None,
        "traffic_unit": "HBM bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)",
        "kernel": "k_score",
        "launches": launches,
        "avg_launch_us": t_launch * 1e6,
        "lookups_per_launch": lookups,
        "valu_lane_instr_per_lookup": valu_per_lookup,
        "counter_profile": os.path.relpath(COUNTERS_FILE, ROOT) if cnt else None,
        "model_ops_per_node_point": MODEL_OPS_PER_NODE_POINT,
        "model_frac": (nodes * args.k * MODEL_OPS_PER_NODE_POINT / (kern_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS
                       if kern_ms > 0 else None),
        "alg_bytes_per_launch": lookups * ALG_BYTES_PER_LOOKUP,
        "alg_gbs": lookups * ALG_BYTES_PER_LOOKUP / t_launch / 1e9 if t_launch > 0 else None,
    }
    line = {
        "metric": METRIC,
        "value": nodes / elapsed,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": len(seeds),
        "warmup": args.warmup,
        "ms_per_step": elapsed / len(seeds) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural city and ray-cast scans)",
        "config": {
            "workload": f"city 500x500x30 m seed 1000 ({len(city.points)} pts), r=1.0 m, l_max=6, "
                        f"{args.k}-pt scans (query seeds 0..{len(seeds) - 1}), roll/pitch +-3 deg, "
                        f"threshold {T}, b={args.batch}, plain batched BnB",
            "mode": "plain",
            "ms_per_localization_mean": elapsed / len(seeds) * 1e3,
            "ms_per_localization_p50": pct(lat, 0.5),
            "ms_per_localization_p99": pct(lat, 0.99),
            "ms_per_localization_found_mean": float(np.mean(found_ms)) if found_ms else None,
            "ms_per_localization_not_found_mean": float(np.mean(lost_ms)) if lost_ms else None,
            "nodes_scored_total": nodes,
            "nodes_expanded_total": sum(r["nodes_expanded"] for r in results),
            "found": f"{sum(r['found'] for r in results)}/{len(seeds)}",
            "success_2m_0p05rad": f"{ok}/{len(seeds)}",
            "parity_vs_oracle": golden_parity(results, seeds, args.k, args.batch),
            "map_build_ms": map_ms,
            "score_kernel_ms_mean": kern_ms / len(seeds),
            "serial_push_ms_mean": sum(r["serial_ms"][0] for r in results) / len(seeds),
            "serial_gather_ms_mean": sum(r["serial_ms"][1] for r in results) / len(seeds),
            "iterations_mean": launches / len(seeds),
        },
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_extra:
        same = lambda rr: sum(a["found"] == b["found"] and a["leaf"] == b["leaf"] and a["score"] == b["score"] and
                              a["nodes_expanded"] == b["nodes_expanded"] for a, b in zip(rr, results))
        for mode, kw in (("persistent", {"persistent": True}), ("graph", {"graph": True}),
                         ("nested_angles", {"nested_angles": True})):
            bbs.localize(gmap, dev[warm_seeds[0] if warm_seeds else 0], lo, hi, T, batch_size=args.batch,
                         workspace=ws, **kw)
            rr, dt = timed_leg(gmap, dev, seeds, lo, hi, T, args.batch, ws, **kw)
            line["config"][mode] = {"ms_per_localization_mean": dt / len(seeds) * 1e3,
                                    "nodes_per_s": sum(r["nodes_scored"] for r in rr) / dt,
                                    "same_result_as_plain": f"{same(rr)}/{len(seeds)}"}
            if mode == "nested_angles":
                # another angular grid (a reading option): its own results, not the plain ones
                line["config"][mode].update({
                    "reading": "angular cells nested top down (option nested_angles), not the default grid",
                    "nodes_scored_total": sum(r["nodes_scored"] for r in rr),
                    "found": f"{sum(r['found'] for r in rr)}/{len(seeds)}",
                    "success_2m_0p05rad": f"{sum(success(r, scans[s].pose) for s, r in zip(seeds, rr))}/{len(seeds)}",
                    "parity_vs_oracle": golden_parity(rr, seeds, args.k, args.batch, "nested")})
            print(f"[bench] {mode}: {line['config'][mode]}", file=sys.stderr, flush=True)
        # achievable memory rates: a streaming read of 1 GiB (HBM) and random
        # 8-byte gathers into a table of the size of the map's level grids
        info = gmap.info()
        grid_bytes = sum(8 * n for n in info["dense_entries"])
        probes = {"stream_1gib": bbs.bandwidth_probe("stream", 1 << 30),
                  "gather_level_grids": bbs.bandwidth_probe("gather", max(grid_bytes, 1 << 16), 1 << 27)}
        roofline["achievable"] = probes
        roofline["alg_frac_of_gather"] = (roofline["alg_gbs"] / probes["gather_level_grids"]["gbs"]
                                          if roofline["alg_gbs"] else None)
        if cnt and t_launch > 0:
            req = cnt["l2_read_req_per_lookup"] * lookups / t_launch
            roofline["l2_read_requests_per_s"] = req
            # one request per 8-byte gather in the probe: its load rate is the achievable request rate
            roofline["l2_frac_of_gather_requests"] = req / (probes["gather_level_grids"]["gbs"] * 1e9 / 8)
        if traffic and t_launch > 0:
            roofline["hbm_gbs"] = traffic["bytes_per_launch"] / t_launch / 1e9
            roofline["hbm_frac_of_stream"] = roofline["hbm_gbs"] / probes["stream_1gib"]["gbs"]
    learned = None
    if not args.no_learned and os.path.exists(WEIGHTS):
        learned = learned_order(gmap, dev, seeds, results, lo, hi, T, args)
        line["config"]["learned"] = learned["summary"]
    if args.details:
        with open(args.details, "w") as f:
            json.dump({"seeds": seeds, "results": results,
                       "learned": learned["results"] if learned else None}, f, indent=1)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(city.points, scans[seeds[0]].points, lo, hi, T, args.batch,
                                            args.cpu_seconds)
        if not args.no_extra:
            line["config"]["indoor"] = indoor_leg(args.cpu_seconds)
    print(json.dumps(line), flush=True)


def learned_order(gmap, dev, seeds, plain, lo, hi, T, args):
    """The same queries with the proposal network's prior (prior-ordered initial
    set and seed beam).  Timed per query: the prior (BEV image and network
    forward on the device) + localization."""
    import numpy as np
    import torch

    import paper_2310_10023_amd as bbs
    from paper_2310_10023_amd import proposal
    net = proposal.Net(max_batch=1, params=np.load(WEIGHTS)["params"])
    ws = bbs.Workspace()
    out = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prior_ms = 0.0
    for s in seeds:
        ta = time.perf_counter()
        logits = net.prior(dev[s])
        prior_ms += (time.perf_counter() - ta) * 1e3
        out.append(bbs.localize(gmap, dev[s], lo, hi, T, batch_size=args.batch, workspace=ws, prior=logits,
                                seed_beam=args.beam))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    same = sum(a["found"] == b["found"] and a["leaf"] == b["leaf"] and a["score"] == b["score"]
               for a, b in zip(out, plain))
    ge = sum(a["score"] >= b["score"] for a, b in zip(out, plain))
    summary = {
        "ms_per_localization_mean": elapsed / len(seeds) * 1e3,
        "prior_ms_mean": prior_ms / len(seeds),
        "nodes_scored_total": sum(r["nodes_scored"] for r in out),
        "nodes_expanded_total": sum(r["nodes_expanded"] for r in out),
        "plain_nodes_expanded_total": sum(r["nodes_expanded"] for r in plain),
        "nodes_per_s": sum(r["nodes_scored"] for r in out) / elapsed,
        "same_result_as_plain": f"{same}/{len(seeds)}",
        "score_at_least_plain": f"{ge}/{len(seeds)}",
        "seeded": sum(r["seeded"] for r in out),
        "beam": args.beam,
    }
    return {"summary": summary, "results": out}


def net_flops_per_image():
    """Multiply-adds x 2 of one forward pass: four 3x3 stride-2 convolutions
    (64x64 input, 1->16->32->64->64 channels) and two FC layers (1024->256,
    256->1088), each one GEMM of output pixels x output channels x (9 x input
    channels)."""
    ch = [1, 16, 32, 64, 64]
    hw, fwd, dgrad = 64, 0, 0
    for i in range(4):
        hw //= 2
        f = 2 * hw * hw * ch[i + 1] * 9 * ch[i]
        fwd += f
        dgrad += f if i > 0 else 0          # no input gradient for the image
    fc = 2 * 1024 * 256 + 2 * 256 * 1088
    return fwd + fc, dgrad + fc


def net_bench(args):
    """The learned proposal's MFMA kernels: one AdamW training step at the
    training batch (forward, input and weight gradients, loss, AdamW), the
    forward pass at batch 1 and 16, and the device prior of a resident city
    scan (BEV image + forward pass).  Synthetic images: the GEMM shapes do not
    depend on their content."""
    import numpy as np
    import torch

    import synth
    from paper_2310_10023_amd import proposal
    rng = np.random.default_rng(0)
    B = args.net_batch
    net = proposal.Net(max_batch=max(256, B), params=np.load(WEIGHTS)["params"])
    imgs = (rng.random((B, 64, 64)) < 0.1).astype(np.uint8) * rng.integers(1, 255, (B, 64, 64), dtype=np.uint8)
    yaw = rng.integers(0, 64, B).astype(np.int32)
    xy = rng.integers(0, 1024, B).astype(np.int32)
    for _ in range(3):
        net.train_step(imgs, yaw, xy, lr=1e-6)
    n_steps = max(5, args.steps)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        net.train_step(imgs, yaw, xy, lr=1e-6)
    step_s = (time.perf_counter() - t0) / n_steps
    fwd_f, back_f = net_flops_per_image()
    train_flops = B * (2 * fwd_f + back_f)       # forward, weight gradient, input gradient
    out = {}
    for b in (1, 16):
        x = imgs[:b]
        net.forward(x)
        t0 = time.perf_counter()
        for _ in range(50):
            net.forward(x)
        out[f"forward_b{b}_ms"] = (time.perf_counter() - t0) / 50 * 1e3
    city = synth.city_scene(1000)
    dev = torch.from_numpy(synth.city_query(city, 0, args.k, voxel=0.5).points).cuda()
    net.prior(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(50):
        net.prior(dev)
    prior_ms = (time.perf_counter() - t0) / 50 * 1e3
    achieved = train_flops / step_s / 1e12
    line = {
        "metric": "proposal network: training step and inference (BF16 MFMA), 1 GPU",
        "value": B / step_s, "unit": "training images/s", "n_gpus": 1, "steps": n_steps, "warmup": 3,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic (random sparse BEV images and labels)",
        "config": {"workload": f"proposal network, training batch {B}, AdamW; forward at batch 1 and 16; "
                               f"device prior of a {args.k}-point city scan",
                   "flops_per_image_forward": fwd_f, "flops_per_training_step": train_flops,
                   "prior_ms": prior_ms, **out},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None,
                     "note": "dense bf16 MFMA peak; the network is small, so each GEMM has few tiles and the step "
                             "is bound by launches and their latency"},
    }
    print(json.dumps(line), flush=True)
    net.close()


def rot_exact_bench(args):
    """The exact rotational bound on the city workload: the map is built with
    the grown tables that the queries' margins need (largest over the
    queries whose margins are all at most 8; a query whose angular grid makes
    child cells drift far from their parent's angle needs more and is
    skipped), then those queries are localized plain and with rot_exact.  One
    JSON line: ms per localization and nodes scored of both, and how many
    results agree."""
    import numpy as np
    import torch

    import paper_2310_10023_amd as bbs
    import synth
    city = synth.city_scene(1000)
    lo, hi = synth.search_range_city()
    T = synth.threshold_95(args.k)
    seeds = list(range(args.steps))
    scans = {s: synth.city_query(city, s, args.k, voxel=0.5) for s in seeds}
    ranges = {s: float(np.sqrt((v.points.astype(np.float64) ** 2).sum(1)).max()) for s, v in scans.items()}
    margins = {s: bbs.rotation_margins(1.0, 6, d, lo, hi, nested_angles=args.nested) for s, d in ranges.items()}
    all_seeds = seeds
    seeds = [s for s in seeds if max(margins[s]) <= 8]
    dmax = max(ranges[s] for s in seeds)
    need = [max(col) for col in zip(*(margins[s] for s in seeds))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gmap = bbs.Map(torch.from_numpy(city.points).cuda(), 1.0, 6, margins=need)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    dev = {s: torch.from_numpy(v.points).cuda() for s, v in scans.items()}
    ws = bbs.Workspace()
    out = {}
    for mode in ("plain", "rot_exact"):
        kw = {"rot_exact": mode == "rot_exact", "batch_size": args.batch, "workspace": ws,
              "nested_angles": args.nested}
        bbs.localize(gmap, dev[seeds[0]], lo, hi, T, **kw)
        res, ms = [], []
        for s in seeds:
            torch.cuda.synchronize()
            ta = time.perf_counter()
            res.append(bbs.localize(gmap, dev[s], lo, hi, T, **kw))
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - ta) * 1e3)
            print(f"[bench] {mode} seed {s}: {ms[-1]:.1f} ms, {res[-1]['nodes_scored']} nodes", file=sys.stderr,
                  flush=True)
        out[mode] = {"ms_mean": float(np.mean(ms)), "ms_p50": pct(ms, 0.5), "nodes_scored_total":
                     sum(r["nodes_scored"] for r in res), "found": sum(r["found"] for r in res),
                     "success_2m_0p05rad": sum(success(r, scans[s].pose) for s, r in zip(seeds, res)),
                     "results": res}
    same = sum(a["found"] == b["found"] and a["score"] == b["score"] and a["leaf"] == b["leaf"]
               for a, b in zip(out["plain"]["results"], out["rot_exact"]["results"]))
    higher = sum(b["score"] > a["score"] for a, b in zip(out["plain"]["results"], out["rot_exact"]["results"]))
    for m in out.values():
        del m["results"]
    line = {
        "metric": "ms per localization, exact rotational bound vs the paper's bound, 1 GPU",
        "value": out["rot_exact"]["ms_mean"], "unit": "ms per localization (rot_exact)", "n_gpus": 1,
        "steps": len(seeds), "warmup": 1, "ms_per_step": out["rot_exact"]["ms_mean"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded procedural city and ray-cast scans)",
        "config": {"workload": f"city seed 1000, {args.k}-pt scans (query seeds {seeds}), b={args.batch}"
                               + (", nested angular grid" if args.nested else ""),
                   "margins": need, "d_max_largest": dmax, "map_build_ms_with_grown_tables": build_ms,
                   "queries_within_margin_8": f"{len(seeds)}/{len(all_seeds)}",
                   "margins_of_skipped": {str(s): margins[s] for s in all_seeds if s not in seeds},
                   "plain": out["plain"], "rot_exact": out["rot_exact"],
                   "same_result": f"{same}/{len(seeds)}", "higher_score_with_exact_bound": higher},
    }
    print(json.dumps(line))


def tuned_bench(args):
    """Autotuned search (a8): b in 1k..64k and the scoring tile picked by
    bbs_autotune on 3 sample queries per scan size, for per-iteration launches
    and for the persistent kernel; the faster of the two is timed on the query
    seeds 0..n-1 against plain launches at b = 10000 (the persistent kernel's
    own best is timed too, for the record)."""
    import numpy as np
    import torch

    import paper_2310_10023_amd as bbs
    import synth
    city = synth.city_scene(1000)
    lo, hi = synth.search_range_city()
    gmap = bbs.Map(torch.from_numpy(city.points).cuda(), 1.0, 6)
    ws = bbs.Workspace()
    out = {}
    tot_nodes, tot_s = 0, 0.0
    b_grid = [1000, 2000, 4000, 8000, 16000, 32000, 64000]
    t_grid = [1024, 2048, 4096, 8192]
    for k in (5000, 10000, 20000):
        T = synth.threshold_95(k)
        tune = [torch.from_numpy(synth.scan_scene(city, 300 + i, k, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048,
                                                  voxel=0.25).points).cuda() for i in range(3)]
        best_l, _ = bbs.autotune(gmap, tune, lo, hi, [T] * 3, b_grid, t_grid, persistent=False)
        best_p, _ = bbs.autotune(gmap, tune, lo, hi, [T] * 3, b_grid, t_grid, persistent=True)
        pick = dict(best_l, persistent=False) if best_l["ms"] <= best_p["ms"] else dict(best_p, persistent=True)
        dev = [torch.from_numpy(synth.scan_scene(city, i, k, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048,
                                                 voxel=0.25).points).cuda() for i in range(args.tuned_queries)]
        res = {}
        for mode, kw in (("plain_b10000", dict(batch_size=10000)),
                         ("tuned", dict(batch_size=pick["batch_size"], score_items=pick["score_items"],
                                        persistent=pick["persistent"])),
                         ("persistent_tuned", dict(batch_size=best_p["batch_size"], score_items=best_p["score_items"],
                                                   persistent=True))):
            bbs.localize(gmap, dev[0], lo, hi, T, workspace=ws, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rr = [bbs.localize(gmap, d, lo, hi, T, workspace=ws, **kw) for d in dev]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            nodes = sum(r["nodes_scored"] for r in rr)
            res[mode] = {"ms_per_localization": dt / len(dev) * 1e3, "nodes_per_s": nodes / dt,
                         "found": f"{sum(r['found'] for r in rr)}/{len(dev)}"}
            if mode == "tuned":
                tot_nodes += nodes
                tot_s += dt
        res["pick"] = pick
        res["persistent_best"] = best_p
        out[str(k)] = res
        print(f"[bench] k={k}: {res}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC + " (autotuned)",
        "value": tot_nodes / tot_s,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": 3 * args.tuned_queries,
        "warmup": 3,
        "ms_per_step": tot_s / (3 * args.tuned_queries) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural city and ray-cast scans)",
        "config": {"workload": f"city seed 1000, scans of 5k/10k/20k pts (query seeds 0..{args.tuned_queries - 1}), "
                               "b, scoring tile and loop form (launches or persistent kernel) autotuned on seeds "
                               "300..302", "per_k": out},
    }
    print(json.dumps(line), flush=True)


def table1_bench(args):
    """Table I of the paper on synthetic maps: the nine combinations of
    processing type (CPU one thread, CPU four threads, GPU), branching
    (translation only, or translation and rotation) and search strategy
    (depth first, best first), on the tiny indoor workload (room, r = 0.5 m,
    l_max = 4) with 1,000-point scans as in the paper's experiments (Sec. IV).
    The GPU runs every query seed; each CPU configuration (the oracle) runs as
    many seeds as fit in --table1-cpu-seconds and reports how many it ran."""
    import numpy as np
    import torch

    import oracle
    import paper_2310_10023_amd as bbs
    import synth
    scene = synth.room_scene(0)
    lo, hi = synth.search_range_room()
    k = args.table1_k
    T = synth.threshold_95(k)
    n = args.table1_queries
    scans = [synth.room_query(scene, s, k) for s in range(n)]
    gmap = bbs.Map(torch.from_numpy(scene.points).cuda(), 0.5, 4)
    omap = oracle.Map(scene.points, 0.5, 4)
    dev = [torch.from_numpy(sc.points).cuda() for sc in scans]
    ws = bbs.Workspace()
    configs = [("c", "gpu", True, "depth_first"), ("f", "gpu", True, "best_first"), ("i", "gpu", False, "best_first"),
               ("a", "cpu1", True, "depth_first"), ("b", "cpu4", True, "depth_first"),
               ("d", "cpu1", True, "best_first"), ("e", "cpu4", True, "best_first"),
               ("g", "cpu1", False, "best_first"), ("h", "cpu4", False, "best_first")]
    rows = {}
    gpu_res = {}
    for name, kind, trans, strat in configs:
        ms, res = [], []
        if kind == "gpu":
            bbs.localize(gmap, dev[0], lo, hi, T, workspace=ws, translation_only=trans, strategy=strat)
            for d in dev:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res.append(bbs.localize(gmap, d, lo, hi, T, workspace=ws, translation_only=trans, strategy=strat))
                torch.cuda.synchronize()
                ms.append((time.perf_counter() - t0) * 1e3)
            gpu_res[(trans, strat)] = res
        else:
            threads = 1 if kind == "cpu1" else 4
            t_end = time.perf_counter() + args.table1_cpu_seconds

            def run():
                for sc in scans:
                    if time.perf_counter() > t_end:
                        break
                    t0 = time.perf_counter()
                    s = oracle.Search(omap, sc.points, lo, hi, translation_only=trans)
                    res.append(s.localize(T, batch=10000, threads=threads, strategy=strat))
                    ms.append((time.perf_counter() - t0) * 1e3)
            if threads == 1:
                with_one_core(run)
            else:
                run()
        ok = sum(success(r, sc.pose) for r, sc in zip(res, scans))
        same = None
        if kind != "gpu" and (trans, strat) in gpu_res:
            keys = ("found", "score", "leaf", "nodes_expanded", "nodes_scored")
            same = f"{sum(all(a[x] == b[x] for x in keys) for a, b in zip(res, gpu_res[(trans, strat)]))}/{len(res)}"
        rows[name] = {"processing": {"cpu1": "CPU single-thread (1 pinned core)", "cpu4": "CPU multi-thread (4 threads)",
                                     "gpu": "GPU"}[kind],
                      "branching": "trans." if trans else "trans. and rot.",
                      "strategy": "DFS" if strat == "depth_first" else "BFS",
                      "queries": len(res), "ms_mean": float(np.mean(ms)) if ms else None,
                      "ms_p50": pct(ms, 0.5), "success_2m_0p05rad": f"{ok}/{len(res)}",
                      "nodes_scored_mean": float(np.mean([r["nodes_scored"] for r in res])) if res else None,
                      "equal_to_gpu_row": same}
        print(f"[bench] table1 ({name}): {rows[name]}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC + " (Table I configurations)",
        "value": rows["i"]["ms_mean"],
        "unit": "ms per localization (configuration (i))",
        "n_gpus": 1,
        "steps": n,
        "warmup": 1,
        "ms_per_step": rows["i"]["ms_mean"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded room and ray-cast scans)",
        "config": {"workload": f"room 20x20x5 m seed 0, r=0.5 m, l_max=4, {k}-pt scans (query seeds 0..{n - 1}), "
                               f"threshold {T}, b=10000", "table1": {c: rows[c] for c in "abcdefghi"}},
    }
    print(json.dumps(line), flush=True)


def stream_bench(args):
    """Stream of queries on the resident city map: scans of 2k-30k points,
    Poisson arrivals at 0.7x the measured service rate of the workers, and a
    saturation run with every query arriving at once."""
    import numpy as np
    import torch

    import paper_2310_10023_amd as bbs
    import synth
    rng = np.random.default_rng(0)
    city = synth.city_scene(1000)
    lo, hi = synth.search_range_city()
    n = args.stream_queries
    ks = rng.integers(2000, 30001, size=n)
    t0 = time.perf_counter()
    scans = [synth.scan_scene(city, 5000 + i, int(ks[i]), z=1.8, rp_deg=3.0, n_beams=64, n_az=2048, voxel=0.25)
             for i in range(n)]
    print(f"[bench] {n} stream scans ready in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    gmap = bbs.Map(torch.from_numpy(city.points).cuda(), 1.0, 6)
    dev = [torch.from_numpy(s.points).cuda() for s in scans]
    thr = [synth.threshold_95(len(s.points)) for s in scans]
    rngs = [(lo, hi)] * n
    # warm up, then saturation: everything arrives at t = 0
    bbs.serve(gmap, dev[:8], rngs[:8], thr[:8], [0.0] * 8, workers=args.stream_workers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, ts, te = bbs.serve(gmap, dev, rngs, thr, [0.0] * n, workers=args.stream_workers)
    sat = time.perf_counter() - t0
    rate = n / sat
    arr = np.cumsum(rng.exponential(1.0 / (0.7 * rate), size=n))
    arr -= arr[0]
    t0 = time.perf_counter()
    res2, ts2, te2 = bbs.serve(gmap, dev, rngs, thr, arr, workers=args.stream_workers)
    wall = time.perf_counter() - t0
    lat = np.sort(te2 - arr) * 1e3
    nodes = sum(r["nodes_scored"] for r in res2)
    line = {
        "metric": METRIC + " (stream)",
        "value": n / wall,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": 8,
        "ms_per_step": wall / n * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural city and ray-cast scans)",
        "config": {
            "workload": f"stream of {n} queries on the city (seed 1000), scans 2k-30k pts, roll/pitch +-3 deg, "
                        f"Poisson arrivals at 0.7x saturation rate, {args.stream_workers} workers, plain batched BnB",
            "saturation_queries_per_s": rate,
            "latency_ms_p50": float(lat[len(lat) // 2]),
            "latency_ms_p99": float(lat[min(len(lat) - 1, int(0.99 * len(lat)))]),
            "nodes_scored_per_s": nodes / wall,
            "found": f"{sum(r['found'] for r in res2)}/{n}",
        },
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
