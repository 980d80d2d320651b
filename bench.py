"""Throughput of exact Density Peaks Clustering on one MI355X.

One step = one dpc_run over the whole point set: bounds, Morton sort, index
build, density, priority keys, dependent points and labels (every step of
the method), with the points already resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="varden2d_10m")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this build runs on one GPU only: the hot path is single-GPU (see DESIGN.md for how it "
              "would shard); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import datagen
    import paper_2305_11335_amd as dpc

    inst = datagen.make(args.workload)
    dev = torch.device("cuda:0")
    P = torch.from_numpy(inst.points).to(dev)
    n = inst.n
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
           torch.empty(n, dtype=torch.int64, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    for _ in range(args.warmup):
        dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / max(args.steps, 1)
    rec = {
        "metric": "points/sec end-to-end exact DPC (10M 2D, 1 GPU)",
        "value": n / (ms / 1000.0),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 coords, exact f64/int64 squared distances",
        "data": "synthetic",
        "config": {"workload": inst.name, "n": n, "d": inst.d, "d_cut": inst.d_cut, "rho_min": inst.rho_min,
                   "delta_min": inst.delta_min, "seed": inst.seed},
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
