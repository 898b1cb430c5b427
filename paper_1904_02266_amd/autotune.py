"""Offline sweep of the work-item sizing (needs the GPU).

For each size class a representative registration is timed with every
candidate (work_item_min, work_items_max) pair, set explicitly in the
parameters, and the fastest pair is written to the tuning table that
cvo_create loads (tuning.json next to this file):

    python -m paper_1904_02266_amd.autotune [--out paper_1904_02266_amd/tuning.json]

Classes (a request uses the first of its kind, cutoff or not, that holds
max(n_src, n_tgt) points):
  brute force  <= 4,096     three planes, 2,000 points, 50 steps
  brute force  <= 65,536    three planes, 16,000 points, 8 steps
  cutoff       <= 12,288    RGB-D pair, 8,000 semi-dense points, 4 x 25 iterations
  cutoff       <= 40,000    RGB-D pair, 30,000 semi-dense points (the 30k benchmark pair)
  cutoff       <= 100,000   RGB-D pair, 60,000 semi-dense points
  cutoff       <= 16,000,000 dense frame, 300,000 random pixels (the headline registration)
Each candidate: one warm-up, then the median of `repeats` registrations
(inputs in HBM).  The sizing changes only how the pair work is cut into
work items (and so how the pair terms are grouped into compensated FP32
partials and FP64 sums), not what is computed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CANDIDATES = [(cmin, cmax) for cmax in (64, 128, 256) for cmin in (16, 32, 64, 128, 256, 512, 1024, 2048)]


def classes():
    from paper_1904_02266_amd import params_planes, params_rgbd, synth
    return [
        dict(cutoff=0, max_points=4096, name="planes-2k", make=lambda: synth.planes_pair(2000, seed=1),
             params=params_planes()),
        dict(cutoff=0, max_points=65536, name="planes-16k", make=lambda: synth.planes_pair(16000, seed=11),
             params=params_planes(max_iters=8)),
        dict(cutoff=1, max_points=12288, name="rgbd-8k", make=lambda: synth.rgbd_pair(8000, 8000, seed=4100),
             params=params_rgbd()),
        dict(cutoff=1, max_points=40000, name="rgbd-30k", make=lambda: synth.rgbd_pair(30000, 30000, seed=2),
             params=params_rgbd()),
        dict(cutoff=1, max_points=100000, name="rgbd-60k", make=lambda: synth.rgbd_pair(60000, 60000, seed=4101),
             params=params_rgbd()),
        dict(cutoff=1, max_points=16000000, name="dense-300k",
             make=lambda: synth.rgbd_pair(300000, 300000, seed=3, select="random"), params=params_rgbd()),
    ]


def time_one(ctx, t, prm, repeats):
    import torch
    ctx.register(*t, prm)
    torch.cuda.synchronize()
    ms = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        ctx.register(*t, prm)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ms))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--only", default="", help="comma-separated class names (default: all)")
    args = ap.parse_args()
    import dataclasses

    import torch
    from paper_1904_02266_amd import Context
    dev = torch.device("cuda:0")
    ctx = Context(0)
    out = []
    for cl in classes():
        if args.only and cl["name"] not in args.only.split(","):
            continue
        p = cl["make"]()
        t = [torch.from_numpy(a).to(dev) for a in (p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat)]
        torch.cuda.synchronize()
        res = []
        for cmin, cmax in CANDIDATES:
            prm = dataclasses.replace(cl["params"], work_item_min=cmin, work_items_max=cmax)
            res.append((time_one(ctx, t, prm, args.repeats), cmin, cmax))
        res.sort()
        best = res[0]
        default = next(r for r in res if r[1] == 256 and r[2] == 64)
        print(f"autotune: {cl['name']}: best work_item_min {best[1]}, work_items_max {best[2]}: {best[0]:.3f} ms "
              f"(default 256/64: {default[0]:.3f} ms)", file=sys.stderr, flush=True)
        out.append({"cutoff": cl["cutoff"], "max_points": cl["max_points"], "work_item_min": best[1],
                    "work_items_max": best[2], "workload": cl["name"], "ms_per_registration": round(best[0], 4),
                    "default_ms_per_registration": round(default[0], 4),
                    "sweep_ms": {f"{r[1]}/{r[2]}": round(r[0], 4) for r in sorted(res, key=lambda r: (r[2], r[1]))}})
    ctx.close()
    doc = {"command": "python -m paper_1904_02266_amd.autotune", "device": torch.cuda.get_device_name(0),
           "note": "per class: the fastest (work_item_min, work_items_max) of the sweep; ms per registration, "
                   "median of the repeats, inputs in HBM",
           "classes": out}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps({"tuning_table": args.out, "classes": len(out)}), flush=True)


if __name__ == "__main__":
    main()
