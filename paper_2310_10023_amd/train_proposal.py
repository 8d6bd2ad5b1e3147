"""Train the learned proposal network on (scan, plain-BnB optimum) pairs.

    python -m paper_2310_10023_amd.train_proposal --maps 50 --scans 400 --out weights.npz

or in shards: `--map-start S --maps M --data-out shard.npz` per shard, then
`--data a.npz,b.npz,... --out weights.npz`.

For every seeded training city (seeds 0.. maps-1; the benchmark city 1000 is
held out) scans are ray-cast from random street poses, localized by the
plain batched branch and bound on the GPU (bbs_serve), and the optimum leaf
gives the labels: the yaw bin of its yaw and the 32 x 32 cell of its
translation in the search box.  The bird's-eye polar image of the scan and the
training steps run in libbbs (BF16 MFMA kernels, AdamW).
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

import paper_2310_10023_amd as bbs  # noqa: E402
from paper_2310_10023_amd import proposal  # noqa: E402

CONV_CH = (1, 16, 32, 64, 64)


def he_init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, flattened in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(4):
        cin, cout = CONV_CH[i], CONV_CH[i + 1]
        parts.append(rng.normal(size=cout * 9 * cin) * math.sqrt(2.0 / (9 * cin)))
        parts.append(np.zeros(cout))
    parts.append(rng.normal(size=256 * 1024) * math.sqrt(2.0 / 1024))
    parts.append(np.zeros(256))
    parts.append(rng.normal(size=1088 * 256) * math.sqrt(2.0 / 256))
    parts.append(np.zeros(1088))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == proposal.param_count()
    return flat


def _scan_worker(args):
    geom, seed, k = args
    boxes, ground, extent, streets = geom
    scene = synth.Scene(points=np.zeros((0, 3), np.float32), boxes=boxes, ground=ground, walls_box=None,
                        extent=extent, streets=streets)
    sc = synth.scan_scene(scene, seed, k, z=1.8, rp_deg=3.0, n_beams=64, n_az=2048, voxel=0.5)
    return sc.points, sc.pose


def make_dataset(map_seeds, scans_per_map, pool, k=10000, bnb_workers=4, log=print):
    """(BEV image, yaw bin, xy cell) of the plain-BnB optimum for `scans_per_map`
    seeded scans of each city in `map_seeds`.  `pool` is a process pool
    created before the GPU is initialised; it ray-casts the scans."""
    lo, hi = synth.search_range_city()
    T = synth.threshold_95(k)
    images, yaws, cells, meta = [], [], [], []
    for ms in map_seeds:
        t0 = time.time()
        city = synth.city_scene(ms)
        gmap = bbs.Map(city.points, 1.0, 6)
        geom = (city.boxes, city.ground, city.extent, city.streets)
        scans = pool.map(_scan_worker, [(geom, 10_000 * ms + i, k) for i in range(scans_per_map)], chunksize=8)
        pts = [s[0] for s in scans]
        res, _, _ = bbs.serve(gmap, pts, [(lo, hi)] * len(pts), [T] * len(pts), [0.0] * len(pts),
                              workers=bnb_workers)
        kept = 0
        for (p, pose), r in zip(scans, res):
            if not r["found"]:
                continue
            images.append(proposal.bev_image(p))
            yaws.append(proposal.yaw_bin(r["pose"][5]))
            cells.append(proposal.xy_cell(r["pose"][0], r["pose"][1], lo, hi))
            meta.append((ms, float(np.hypot(*(np.array(r["pose"][:2]) - pose[:2])))))
            kept += 1
        gmap.close()
        del city
        log(f"[data] map {ms}: {kept}/{len(pts)} localized in {time.time() - t0:.1f} s")
    return np.stack(images), np.array(yaws, np.int32), np.array(cells, np.int32), meta


def evaluate(net, images, yaw, xy, batch=256):
    """Held-out metrics: mean loss terms are not needed here, only how often
    the true yaw bin / translation cell is among the top-k logits."""
    hits = {"yaw_top1": 0, "yaw_top4": 0, "yaw_top8": 0, "xy_top1": 0, "xy_top16": 0}
    for b0 in range(0, len(images), batch):
        out = net.forward(images[b0:b0 + batch])
        ry = np.argsort(-out[:, :64], axis=1)
        rc = np.argsort(-out[:, 64:], axis=1)
        ty, tc = yaw[b0:b0 + batch], xy[b0:b0 + batch]
        for k in (1, 4, 8):
            hits[f"yaw_top{k}"] += int(np.sum(np.any(ry[:, :k] == ty[:, None], axis=1)))
        for k in (1, 16):
            hits[f"xy_top{k}"] += int(np.sum(np.any(rc[:, :k] == tc[:, None], axis=1)))
    n = max(len(images), 1)
    return {k: v / n for k, v in hits.items()}


def train(images, yaw, xy, epochs=40, batch=128, lr=2e-3, weight_decay=1e-4, seed=0, val=None, init=None, log=print):
    rng = np.random.default_rng(seed)
    net = proposal.Net(max_batch=max(batch, 256), params=he_init(seed) if init is None else init)
    n = len(images)
    steps = 0
    total_steps = max(1, epochs * (n // batch))
    for ep in range(epochs):
        perm = rng.permutation(n)
        # yaw augmentation: rotating the scan by whole azimuth bins shifts the image
        # columns and the yaw label together (the label is the map-frame yaw of the
        # sensor, the image is in the sensor frame: a sensor-frame rotation by s bins
        # is a yaw change of -s bins)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            shift = rng.integers(0, 64, size=len(idx))
            img = np.stack([np.roll(images[i], s, axis=1) for i, s in zip(idx, shift)])
            y = (yaw[idx] - shift) % 64
            cur_lr = lr * 0.5 * (1 + math.cos(math.pi * steps / total_steps))
            loss, _ = net.train_step(img, y, xy[idx], lr=cur_lr, weight_decay=weight_decay)
            tot += loss
            cnt += 1
            steps += 1
        msg = f"[train] epoch {ep}: loss {tot / max(cnt, 1):.3f}"
        if val is not None and (ep % 5 == 4 or ep == epochs - 1):
            msg += " val " + json.dumps({k: round(v, 3) for k, v in evaluate(net, *val).items()})
        log(msg)
    return net.get_params(), (evaluate(net, *val) if val is not None else None)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--maps", type=int, default=50)
    ap.add_argument("--map-start", type=int, default=0, help="first training city seed")
    ap.add_argument("--scans", type=int, default=400)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=None, help="trained parameters (.npz)")
    ap.add_argument("--data", default=None,
                    help="comma-separated cached pair files (.npz) to train on instead of generating pairs")
    ap.add_argument("--data-out", default=None, help="write the generated pairs here (.npz)")
    ap.add_argument("--init", default=None, help="start from these parameters (.npz) instead of He-normal weights")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--val-maps", type=int, default=5,
                    help="the last N training cities of the data are held out for validation")
    args = ap.parse_args()
    if not args.out and not args.data_out:
        ap.error("nothing to do: give --out and/or --data-out")
    # the ray-casting workers are forked before anything touches the GPU
    pool = None if args.data else mp.get_context("fork").Pool(args.workers)
    import torch
    torch.cuda.set_device(0)
    t0 = time.time()
    if args.data:
        parts = [np.load(f) for f in args.data.split(",")]
        images = np.concatenate([d["images"] for d in parts])
        yaw = np.concatenate([d["yaw"] for d in parts])
        xy = np.concatenate([d["xy"] for d in parts])
        map_seed = np.concatenate([d["map_seed"] for d in parts])
    else:
        seeds = range(args.map_start, args.map_start + args.maps)
        images, yaw, xy, meta = make_dataset(seeds, args.scans, pool, log=lambda m: print(m, flush=True))
        map_seed = np.array([m[0] for m in meta], np.int32)
        pool.close()
        pool.join()
        if args.data_out:
            np.savez_compressed(args.data_out, images=images, yaw=yaw, xy=xy,
                                map_seed=np.array([m[0] for m in meta], np.int32),
                                xy_err=np.array([m[1] for m in meta], np.float64))
    print(f"[data] {len(images)} pairs in {time.time() - t0:.1f} s", flush=True)
    if not args.out:
        return
    held = np.unique(map_seed)[-args.val_maps:] if args.val_maps > 0 else np.zeros(0, np.int32)
    is_val = np.isin(map_seed, held)
    val = (images[is_val], yaw[is_val], xy[is_val]) if is_val.any() else None
    print(f"[train] {int((~is_val).sum())} training pairs, {int(is_val.sum())} held-out pairs "
          f"(cities {held.tolist()})", flush=True)
    init = np.load(args.init)["params"] if args.init else None
    params, val_metrics = train(images[~is_val], yaw[~is_val], xy[~is_val], epochs=args.epochs, lr=args.lr, val=val,
                                init=init, log=lambda m: print(m, flush=True))
    np.savez_compressed(args.out, params=params,
                        info=json.dumps({"pairs": int((~is_val).sum()), "held_out_pairs": int(is_val.sum()),
                                         "held_out_cities": held.tolist(), "epochs": args.epochs,
                                         "held_out_metrics": val_metrics, "init": bool(args.init),
                                         "data": args.data or f"cities {args.map_start}..{args.map_start + args.maps - 1}"}))
    print(f"[train] wrote {args.out} after {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
