"""Calibrate each workload's d_cut and write datagen/params.json.

Uses only the oracle (its per-query density, Section 3 Definition 1) on a
seeded sample of query points drawn against the full point set, split over
worker processes.  The radius is the smallest integer d_cut (to within 2%)
whose sampled median (or mean) density reaches the workload's target: a
doubling search brackets it, then bisection narrows the bracket.  Integers
keep the threshold d_cut^2 exact.  Run once:

    python oracle/calibrate_dcut.py [workload ...]
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
import oracle  # noqa: E402

SAMPLES = {"median": 401, "mean": 1000}


def stat(kind, rho):
    return float(np.median(rho)) if kind == "median" else float(np.mean(rho))


_PTS = None


def _init(name):
    global _PTS
    _PTS = datagen.make(name, d_cut=1.0).points


def _chunk(args):
    T, q = args
    return oracle.density_at(_PTS, T, q)


def calibrate(name: str, workers: int = 8) -> dict:
    spec = datagen.WORKLOADS[name]
    kind, target = spec["target"]
    pts = datagen.make(name, d_cut=1.0).points
    rng = datagen.rng_for(10_000 + spec["seed"])
    q = rng.choice(pts.shape[0], size=SAMPLES[kind], replace=False).astype(np.int64)
    t0 = time.time()
    with ProcessPoolExecutor(workers, initializer=_init, initargs=(name,)) as ex:
        def sampled(r):
            parts = list(ex.map(_chunk, [(r * r, c) for c in np.array_split(q, workers)]))
            rho = np.concatenate(parts)
            print(f"  {name}: d_cut {r} -> {kind} rho {stat(kind, rho):.2f}  ({time.time() - t0:.0f}s)",
                  flush=True)
            return rho

        hi = 1
        while stat(kind, sampled(hi)) < target:
            hi *= 2
        lo = hi // 2
        while hi - lo > max(1, hi // 50):
            mid = (lo + hi) // 2
            if stat(kind, sampled(mid)) >= target:
                hi = mid
            else:
                lo = mid
        rho = sampled(hi)
    return {"d_cut": float(hi), "target": [kind, target], "sampled_stat": stat(kind, rho),
            "sample_size": int(q.shape[0]), "sample_rho_p50": float(np.median(rho)),
            "sample_rho_mean": float(np.mean(rho)), "sample_rho_max": int(rho.max())}


def main(names):
    path = os.path.join(ROOT, "datagen", "params.json")
    params = {}
    if os.path.exists(path):
        with open(path) as f:
            params = json.load(f)
    for name in names:
        params[name] = calibrate(name)
        with open(path, "w") as f:
            json.dump(params, f, indent=1, sort_keys=True)
        print(name, params[name], flush=True)


if __name__ == "__main__":
    todo = sys.argv[1:] or [k for k, v in datagen.WORKLOADS.items() if "target" in v]
    main(todo)
