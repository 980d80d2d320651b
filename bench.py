"""Throughput of exact Density Peaks Clustering on one MI355X.

One step = one dpc_run over the whole point set: coordinate bounds, k-d tree
build, density, priority keys, dependent points and labels (every step of the
method), with the points already resident in HBM.  The workload is the
10-million-point 2-D variable-density set (varden2d_10m, see datagen).

Prints one JSON line: throughput, the roofline of the dominant kernel (its
average GPU time measured with HIP events on the launch stream during the
timed steps; its algorithmic work from one extra instrumented run outside the
timed region), the plain O(n^2) CPU oracle timed on a bounded sample
("cpu_baseline") and the multithreaded CPU k-d tree version on the whole
workload with all allowed host threads ("cpu_parallel", outputs compared with
the GPU's).

A second measurement, "batched", runs the 512-instance workload (n
log-uniform in [1e3, 2e5], d in {2, 3, 5, 8}) as one dpc_batch_run per step
and, for comparison, as a loop of per-instance dpc_run calls on one stream
and on four streams (one host thread each); outputs of the three are
compared bit for bit.

A third, "served", replays a Poisson arrival stream (200 requests/s for 60 s
after a 5 s warm-up, n log-uniform in [1e3, 1e6], d = 3, uniform or
clustered; requests drawn from a resident pool of 256 instances) through a
dpc_server (HBM budget 200 GB) and reports p50/p99 latency (completion minus
scheduled arrival) and throughput,
beside the same trace run as plain per-request dpc_run calls in arrival
order; each pool instance's served outputs are compared with its dpc_run
outputs.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-batch]
                    [--no-serve] [--serve-seconds S]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/sec end-to-end exact DPC (10M 2D, 1 GPU); batched instances/s; p99 ms"
# MI355X published peaks
PEAK_LANE_TOPS = 39.3            # VALU lane-instructions/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_HBM_GBPS = 8000.0
ORACLE_SAMPLE = 32768            # points of the CPU-baseline sample
CONFIG2 = ("mix3d_10m", "aniso8d_10m")  # the 10M-point 3-D and 8-D workloads


def ops_per_pair(d: int, narrow: bool) -> float:
    """VALU lane-instructions of one exact pair test (one query against one
    point) on the cheapest exact path the kernels use, counted in this
    build's gfx950 assembly: on narrow leaves, per packed word of two axes a
    16-bit subtract and a dot product, then the count. Up to two dimensions
    each point's sign bit is funnel-shifted into a word and a batch of 16 is
    counted with one population count (17 instructions per 16 points:
    3.0625 in 2-D); from three dimensions on, batches of two take three
    (2 * ceil(d/2) + 1.5).  In exact doubles: d subtractions, one multiply,
    d - 1 fused multiply-adds and about two instructions to compare and keep
    the result (2d + 2)."""
    if not narrow:
        return 2 * d + 2
    return 2 * ((d + 1) // 2) + (17 / 16 if d <= 2 else 1.5)


def alg_bytes_per_point(d: int) -> int:
    """Compulsory HBM bytes per point of density + dependent + labels: read
    the coordinates twice (4d each), write rho (4), read rho for the keys (4),
    write dep and delta2 (12), read rho, dep, delta2 for the labels (16) and
    write the label (4): 8d + 40."""
    return 8 * d + 40


def arith_of(points) -> str:
    """Which exact arithmetic the library uses for these points (its rule)."""
    import numpy as np

    span = points.max(axis=0).astype(np.int64) - points.min(axis=0).astype(np.int64)
    s = sum(int(w) * int(w) for w in span)
    return "f64" if s < (1 << 53) else "int64"


def _profiled(path: str, kernel: str):
    """The record of `kernel` in a committed rocprofv3 counter summary, or
    None if there is none or the kernel's sources changed since the counters
    were taken."""
    import hashlib

    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    k = prof.get("kernels", {}).get(kernel)
    if k is None:
        return None
    h = hashlib.sha256()
    for src in k["sources"]:
        with open(os.path.join(ROOT, "paper_2305_11335_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    return k if h.hexdigest() == k["source_sha256"] else None


def profiled_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` (FETCH_SIZE and WRITE_SIZE, scaled by
    a plain copy's readings) from the committed summary, or None."""
    k = _profiled(os.path.join(ROOT, "profiles", f"traversal_{workload}_hbm_bytes.json"), kernel)
    return None if k is None else k["bytes"]


def profiled_valu(workload: str, kernel: str):
    """VALU wave-instructions per launch of `kernel` (SQ_INSTS_VALU) from the
    committed summary, or None."""
    k = _profiled(os.path.join(ROOT, "profiles", f"traversal_{workload}_valu.json"), kernel)
    return None if k is None else k["valu_wave_insts"]


def roofline(inst, stage_ms: dict, work: dict, ms_step: float) -> dict:
    """The dominant traversal kernel against the integer-ALU roofline, plus
    the whole step against the HBM roofline (SURVEY's compulsory bytes).

    achieved: the kernel's pair tests (counted by the instrumented kernels)
    times the VALU lane-instructions of one exact pair test on its cheapest
    path, over its average time (HIP events on the launch stream during the
    timed steps).  valu_issue_frac: the VALU instructions the kernel really
    issues (a committed SQ_INSTS_VALU profile) over the same time and peak,
    when the profile matches the sources."""
    dom = max(("density", "dependent"), key=lambda k: stage_ms[k])
    pairs = work["density_pairs"] if dom == "density" else work["dependent_pairs"]
    d = inst.d
    narrow = dom == "density" and arith_of(inst.points) == "f64"
    ops = ops_per_pair(d, narrow)
    kernel_s = stage_ms[dom] / 1000.0
    achieved = pairs * ops / kernel_s / 1e12
    valu = profiled_valu(inst.name, f"k_{dom}")
    alg = alg_bytes_per_point(d) * inst.n
    return {"bound": "alu", "kernel": f"k_{dom}", "achieved": achieved, "peak": PEAK_LANE_TOPS,
            "unit": "T VALU lane-ops/s", "frac": achieved / PEAK_LANE_TOPS,
            "traffic": profiled_traffic(inst.name, f"k_{dom}"),
            "kernel_ms": stage_ms[dom], "pair_tests_per_launch": pairs, "lane_ops_per_pair_test": ops,
            "pair_test_path": "packed 16-bit narrow leaf" if narrow else "exact double",
            "valu_issue_frac": None if valu is None else valu * 64 / kernel_s / (PEAK_LANE_TOPS * 1e12),
            "hbm_step": {"alg_bytes": alg, "achieved_GBps": alg / (ms_step / 1000.0) / 1e9,
                         "peak_GBps": PEAK_HBM_GBPS, "frac": alg / (ms_step / 1000.0) / 1e9 / PEAK_HBM_GBPS,
                         "target_frac": 0.40}}


def cpu_baseline(inst) -> dict:
    """The oracle (single-threaded C, O(n^2)) on the first ORACLE_SAMPLE points."""
    import numpy as np

    import oracle

    m = min(ORACLE_SAMPLE, inst.n)
    pts = np.ascontiguousarray(inst.points[:m])
    d_cut = inst.d_cut * (inst.n / m) ** (1.0 / inst.d)  # same expected density as the full set
    oracle.run(pts[:256], d_cut, inst.rho_min, inst.delta_min)  # load the library
    t0 = time.perf_counter()
    oracle.run(pts, d_cut, inst.rho_min, inst.delta_min)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} points of {inst.name} (input order is a seeded shuffle), d_cut scaled by "
                      f"(n/m)^(1/d) to {d_cut:.3f} for the same expected density; whole method, one thread, "
                      f"{dt:.2f} s"}


def cpu_parallel(inst, gpu_out) -> dict:
    """The multithreaded CPU baseline (k-d tree, all allowed host threads) on
    the whole workload; its outputs must equal the GPU's."""
    import numpy as np

    import cpu_baseline

    threads = cpu_baseline.threads_available()
    t0 = time.perf_counter()
    got = cpu_baseline.run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min, threads=threads)
    dt = time.perf_counter() - t0
    same = all(np.array_equal(a, b.cpu().numpy()) for a, b in zip(got, gpu_out))
    return {"value": inst.n / dt, "unit": "points/s", "cores": threads, "kind": "cpu_kdtree_multithreaded",
            "sample": f"whole {inst.name} ({inst.n} points), one run, {dt:.2f} s",
            "outputs_identical_to_gpu": bool(same)}


def single_workload(torch, dpc, datagen, name: str, steps: int, warmup: int) -> dict:
    """One dpc_run per step on another single workload (the 10M-point 3-D
    and 8-D sets): time per step, per-step GPU times, work counters and the
    roofline of its dominant kernel, like the headline."""
    inst = datagen.make(name)
    dev = torch.device("cuda:0")
    P = torch.from_numpy(inst.points).to(dev)
    n = inst.n
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
           torch.empty(n, dtype=torch.int64, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, out=out, stream=stream)
    torch.cuda.synchronize()
    stage_ms = {k: 0.0 for k in dpc.STAGES}
    t0 = time.perf_counter()
    for _ in range(steps):
        dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, out=out, stream=stream, time_stages=True)
        for k, v in dpc.last_stats()["stage_ms"].items():
            stage_ms[k] += v
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    stage_ms = {k: v / steps for k, v in stage_ms.items()}
    dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, out=out, stream=stream, count_work=True)
    work = dpc.last_stats()
    torch.cuda.synchronize()
    return {"workload": name, "n": n, "d": inst.d, "d_cut": inst.d_cut, "steps": steps, "ms_per_step": ms,
            "points_per_s": n / (ms / 1000.0), "stage_ms": stage_ms,
            "work": {k: work[k] for k in dpc.WORK_FIELDS}, "roofline": roofline(inst, stage_ms, work, ms)}


def batched(torch, dpc, datagen, steps: int, trace_only: bool = False) -> dict:
    """Instances/s of the batched workload: one dpc_batch_run per step against
    per-instance dpc_run loops (one stream; four streams driven by one host
    thread each).  Inputs and outputs are resident; the three forms must give
    identical outputs.  Before timing, the leaf size of each dimension is
    autotuned on that dimension's largest instance.  trace_only: only the
    timed dpc_batch_run calls (for a kernel trace of them)."""
    insts = datagen.batch_instances()
    dev = torch.device("cuda:0")
    pts = [torch.from_numpy(x.points).to(dev) for x in insts]
    probs = [(p, x.d_cut, x.rho_min, x.delta_min) for p, x in zip(pts, insts)]
    total = sum(x.n for x in insts)
    tuned = {}
    for d in sorted({x.d for x in insts}):
        k = max((i for i, x in enumerate(insts) if x.d == d), key=lambda i: insts[i].n)
        r = dpc.autotune(*probs[k])
        tuned[str(d)] = {"instance_n": insts[k].n, "ms_leaf16": r["ms"][16], "ms_leaf32": r["ms"][32],
                         "ms_leaf64": r["ms"][64],
                         "leaf_points": r["chosen"]}
    B = dpc.Batch(probs)
    B.run()  # warm-up (pool growth, code loading)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    if trace_only:
        return {"workload": "batch512", "instances": len(insts), "points": total, "steps": steps,
                "ms_per_batch": t_batch * 1000.0, "instances_per_s": len(insts) / t_batch, "autotuned": tuned}

    outs = [tuple(torch.empty_like(t) for t in r) for r in B.results]

    def loop(streams):
        def work(k, s):
            with torch.cuda.stream(s):
                for i in range(k, len(probs), len(streams)):
                    p, dc, rm, dm = probs[i]
                    dpc.run(p, dc, rm, dm, out=outs[i], stream=s)
            s.synchronize()

        if len(streams) == 1:
            work(0, streams[0])
            return
        th = [threading.Thread(target=work, args=(k, s)) for k, s in enumerate(streams)]
        for t in th:
            t.start()
        for t in th:
            t.join()

    timings = {}
    for ns in (1, 4):
        streams = [torch.cuda.Stream() for _ in range(ns)]
        loop(streams)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loop(streams)
        torch.cuda.synchronize()
        timings[ns] = time.perf_counter() - t0
        for r, o in zip(B.results, outs):
            for a, b in zip(r, o):
                if not torch.equal(a, b):
                    raise RuntimeError("batched and per-instance outputs differ")
    # the same batch recorded once and replayed as a HIP graph (all on one
    # stream: no host work, no library streams)
    s = torch.cuda.Stream()
    gouts = [tuple(torch.empty_like(t) for t in r) for r in B.results]
    with dpc.BatchPlan(probs, outs=gouts, stream=s) as plan:
        plan.capture(s)
        plan.launch(s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.launch(s)
        s.synchronize()
        t_graph = (time.perf_counter() - t0) / steps
        graph_ok = plan.status(s) == 0
    for r, o in zip(B.results, gouts):
        for a, b in zip(r, o):
            if not torch.equal(a, b):
                raise RuntimeError("graph replay and batched outputs differ")
    return {"workload": "batch512", "instances": len(insts), "points": total,
            "dims": sorted({x.d for x in insts}), "steps": steps, "autotuned": tuned,
            "plan_graph_ms_per_batch": t_graph * 1000.0, "plan_graph_instances_per_s": len(insts) / t_graph,
            "plan_status_ok": bool(graph_ok),
            "instances_per_s": len(insts) / t_batch, "ms_per_batch": t_batch * 1000.0,
            "points_per_s": total / t_batch,
            "loop_1stream_instances_per_s": len(insts) / timings[1],
            "loop_4streams_instances_per_s": len(insts) / timings[4],
            "speedup_vs_best_loop": min(timings.values()) / t_batch,
            "outputs_identical": True}


def served(torch, dpc, pool, pts, seconds: float, warm: float, rate: float = 200.0,
           budget: int = 200 * 10**9, seed: int = 55, slots: int = 2, max_batch: int = 64, plain: bool = True) -> dict:
    """p50/p99 latency and throughput of a Poisson request stream, through the
    server and through plain per-request dpc_run calls (same trace).  pool:
    the request instances; pts: their points on the device."""
    import queue

    import numpy as np

    rng = np.random.default_rng(seed)
    horizon = warm + seconds
    gaps = rng.exponential(1.0 / rate, size=int(rate * horizon * 1.5) + 16)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < horizon]
    which = rng.integers(0, len(pool), size=len(arrivals))
    first = {}  # pool entry -> outputs of its first served request
    for k, w in enumerate(which):
        first.setdefault(int(w), k)

    def replay(submit, collect):
        """Submits at the scheduled times from one thread; collect() runs in
        this one, in submission order.  Returns (arrival_ns, done_ns) per request."""
        q = queue.Queue()
        t0 = time.monotonic_ns() + 50_000_000
        sched = [t0 + int(a * 1e9) for a in arrivals]

        def producer():
            for k, w in enumerate(which):
                dt = (sched[k] - time.monotonic_ns()) / 1e9
                if dt > 0:
                    time.sleep(dt)
                q.put((k, submit(k, int(w))))
            q.put(None)

        th = threading.Thread(target=producer)
        th.start()
        done = [0] * len(arrivals)
        while True:
            item = q.get()
            if item is None:
                break
            k, h = item
            done[k] = collect(k, h)
        th.join()
        return sched, done

    def stats(sched, done, nbytes=None):
        lat = []
        pts_done = 0
        t_lo = sched[0] + int(warm * 1e9)
        for k in range(len(sched)):
            if sched[k] >= t_lo:
                lat.append((done[k] - sched[k]) / 1e6)
                pts_done += pool[int(which[k])].n
        lat = np.array(lat)
        span = (max(done) - t_lo) / 1e9
        return {"requests": len(lat), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "requests_per_s": len(lat) / span,
                "points_per_s": pts_done / span}

    # the server: outputs per request (kept for the pool entries' first requests)
    outs = {}
    with dpc.Server(hbm_budget_bytes=budget, slots=slots, max_batch=max_batch) as srv:
        def submit_srv(k, w):
            x = pool[w]
            t, res = srv.submit(pts[w], x.d_cut, x.rho_min, x.delta_min)
            if first[w] == k:
                outs[w] = res
            return t

        sched, done = replay(submit_srv, lambda k, t: srv.wait(t)["done_ns"])
        sst = srv.stats()
    rec = {"workload": "served_poisson200_3d", "rate_req_per_s": rate, "seconds": seconds, "warmup_s": warm,
           "pool_instances": len(pool), "hbm_budget_bytes": budget, "slots": slots, "max_batch": max_batch,
           "server": stats(sched, done),
           "server_stats": {k: sst[k] for k in ("batches", "max_batch_seen", "max_slots_busy", "max_admitted_bytes",
                                                "max_workspace_bytes", "over_footprint")}}

    # plain per-request dpc_run calls on one stream, in arrival order
    s = torch.cuda.Stream()

    def submit_plain(k, w):
        return w

    def collect_plain(k, w):
        x = pool[w]
        dpc.run(pts[w], x.d_cut, x.rho_min, x.delta_min, stream=s)
        s.synchronize()
        return time.monotonic_ns()

    if plain:
        sched, done = replay(submit_plain, collect_plain)
        rec["plain_loop"] = stats(sched, done)
    for w, res in outs.items():
        x = pool[w]
        alone = dpc.run(pts[w], x.d_cut, x.rho_min, x.delta_min)
        for a, b in zip(res, alone):
            if not torch.equal(a, b):
                raise RuntimeError("served and alone outputs differ")
    torch.cuda.synchronize()
    rec["outputs_identical_to_alone"] = True
    return rec


def planned(torch, dpc, pool, pts, calls: int = 200) -> dict:
    """Per-call latency of one served-size instance: dpc_run against a plan
    replayed eagerly and as a HIP graph (each call waited for)."""
    import numpy as np

    x, P = pool[0], pts[0]
    s = torch.cuda.Stream()
    res = {"workload": "served_3d_instance", "n": int(x.points.shape[0]), "d": int(x.points.shape[1]),
           "calls": calls}
    with torch.cuda.stream(s):
        ref = [t.cpu() for t in dpc.run(P, x.d_cut, x.rho_min, x.delta_min, stream=s)]

    def timed(call):
        lat = []
        for _ in range(10):
            call()
        s.synchronize()
        for _ in range(calls):
            t0 = time.perf_counter()
            call()
            s.synchronize()
            lat.append((time.perf_counter() - t0) * 1000.0)
        return {"p50_ms": float(np.percentile(lat, 50)), "mean_ms": float(np.mean(lat))}

    res["run"] = timed(lambda: dpc.run(P, x.d_cut, x.rho_min, x.delta_min, stream=s))
    with dpc.Plan(P, x.d_cut, x.rho_min, x.delta_min, stream=s) as plan:
        res["plan_replay"] = timed(lambda: plan.launch(s))
        same = all(torch.equal(a.cpu(), b) for a, b in zip(plan.out, ref))
        plan.capture(s)
        res["plan_graph"] = timed(lambda: plan.launch(s))
        same = same and all(torch.equal(a.cpu(), b) for a, b in zip(plan.out, ref)) and plan.status(s) == 0
    res["outputs_identical"] = bool(same)
    return res


def backend(torch, dpc, inst, P, want, runs: int = 3, **which) -> dict:
    """The whole method with another dependent-point backend (fenwick=True:
    the Fenwick tree of Algorithm 2; pst=True: the priority-search k-d tree
    with one point per node) on the headline workload (per-step GPU times from
    HIP events), outputs compared with the default k-d tree's."""
    got = dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, **which)
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(got, want))
    total, dep = [], []
    for _ in range(runs):
        t0 = time.perf_counter()
        dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, out=got, time_stages=True, **which)
        st = dpc.last_stats()["stage_ms"]
        torch.cuda.synchronize()
        total.append((time.perf_counter() - t0) * 1000.0)
        dep.append(st["priority"] + st["dependent"])
    total.sort()
    dep.sort()
    return {"workload": inst.name, "runs": runs, "ms_per_step": total[len(total) // 2],
            "dependent_ms": dep[len(dep) // 2], "points_per_s": inst.n / (total[len(total) // 2] / 1000.0),
            "outputs_identical_to_default_tree": bool(same)}


def transfers(torch, inst, ms_step: float, reps: int = 5) -> dict:
    """Host-device copies around one step (context only: the library takes
    device pointers, so they are not part of `value`): the points in from
    pinned host memory, the four outputs back to pinned host memory."""
    import numpy as np

    n, d = inst.n, inst.d
    h_pts = torch.empty((n, d), dtype=torch.int32, pin_memory=True)
    h_pts.copy_(torch.from_numpy(np.ascontiguousarray(inst.points)))
    d_pts = torch.empty((n, d), dtype=torch.int32, device="cuda:0")
    d_out = [torch.empty(n, dtype=t, device="cuda:0") for t in (torch.int32, torch.int32, torch.int64, torch.int32)]
    h_out = [torch.empty(n, dtype=t.dtype, pin_memory=True) for t in d_out]
    torch.cuda.synchronize()

    def timed(fn):
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) * 1000.0)
        return best

    h2d = timed(lambda: d_pts.copy_(h_pts, non_blocking=True))
    d2h = timed(lambda: [h.copy_(t, non_blocking=True) for h, t in zip(h_out, d_out)])
    in_b = n * d * 4
    out_b = n * (4 + 4 + 8 + 4)
    return {"h2d_ms": h2d, "h2d_GBps": in_b / h2d / 1e6, "d2h_ms": d2h, "d2h_GBps": out_b / d2h / 1e6,
            "pcie_inclusive_points_per_s": n / ((h2d + ms_step + d2h) / 1000.0),
            "note": "best of %d; pinned host buffers; not part of value" % reps}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="varden2d_10m")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip both CPU baselines")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-workload measurement")
    ap.add_argument("--no-config2", action="store_true", help="skip the 10M-point 3-D and 8-D workloads")
    ap.add_argument("--config2-steps", type=int, default=5)
    ap.add_argument("--no-fenwick", action="store_true",
                    help="skip the measurements of the other dependent-point backends")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true", help="skip the served-workload measurement")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-pool", type=int, default=256, help="distinct request instances")
    ap.add_argument("--batch-trace", action="store_true",
                    help="run only the batched workload's timed calls (for a kernel trace of them)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import datagen
    import paper_2305_11335_amd as dpc

    if args.batch_trace:
        print(json.dumps({"batched": batched(torch, dpc, datagen, args.batch_steps, trace_only=True)}), flush=True)
        return 0
    inst = datagen.make(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = torch.from_numpy(inst.points).to(dev)
    n, d = inst.n, inst.d
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
           torch.empty(n, dtype=torch.int64, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream()

    def step(**kw):
        dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, out=out, stream=stream, **kw)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stage_ms = {k: 0.0 for k in dpc.STAGES}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(time_stages=True)
        for k, v in dpc.last_stats()["stage_ms"].items():
            stage_ms[k] += v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / max(args.steps, 1)
    stage_ms = {k: v / max(args.steps, 1) for k, v in stage_ms.items()}

    # work of the two traversal kernels, from one instrumented run (not timed)
    step(count_work=True)
    work = dpc.last_stats()
    torch.cuda.synchronize()

    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # dominant kernel: the longer of the two traversals (each stage is one kernel)
    roof = roofline(inst, stage_ms, work, ms)

    rec = {
        "metric": METRIC,
        "value": n / (ms / 1000.0),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "exact integer (i16 dot products, i24 box tests, f64 holding integers)",
        "data": "synthetic (seeded generator, see datagen)",
        "config": {"workload": inst.name, "n": n, "d": d, "d_cut": inst.d_cut, "rho_min": inst.rho_min,
                   "delta_min": inst.delta_min, "seed": inst.seed},
        "stage_ms": stage_ms,
        "work": {k: work[k] for k in dpc.WORK_FIELDS},
        "roofline": roof,
    }
    rec["transfers"] = transfers(torch, inst, ms)
    if not args.no_config2:
        rec["config2"] = {}
        for name in CONFIG2:
            print(f"bench: {name}", file=sys.stderr, flush=True)
            rec["config2"][name] = single_workload(torch, dpc, datagen, name, args.config2_steps, 1)
    if not args.no_fenwick:
        print("bench: Fenwick-tree dependent backend", file=sys.stderr, flush=True)
        rec["fenwick"] = backend(torch, dpc, inst, P, out, fenwick=True)
        rec["fenwick"]["default_tree_dependent_ms"] = stage_ms["priority"] + stage_ms["dependent"]
        print("bench: priority-search k-d tree dependent backend", file=sys.stderr, flush=True)
        rec["priority_search_tree"] = backend(torch, dpc, inst, P, out, pst=True)
        rec["priority_search_tree"]["default_tree_dependent_ms"] = stage_ms["priority"] + stage_ms["dependent"]
    if not args.no_batch:
        print("bench: batched workload", file=sys.stderr, flush=True)
        rec["batched"] = batched(torch, dpc, datagen, args.batch_steps)
    if not args.no_serve:
        print(f"bench: served workload ({args.serve_warmup + args.serve_seconds:.0f} s, twice)", file=sys.stderr,
              flush=True)
        pool = datagen.served_instances(count=args.serve_pool)
        pts = [torch.from_numpy(x.points).to(dev) for x in pool]
        rec["served"] = served(torch, dpc, pool, pts, args.serve_seconds, args.serve_warmup)
        # the same pool offered faster than per-request calls can serve it
        print("bench: served workload under overload (1500 requests/s, 7 s, twice)", file=sys.stderr, flush=True)
        rec["served_overload"] = served(torch, dpc, pool, pts, 6.0, 1.0, rate=1500.0, seed=56)
        rec["served_overload"]["workload"] = "served_poisson1500_3d"
        print("bench: per-call latency, dpc_run against plans", file=sys.stderr, flush=True)
        rec["planned"] = planned(torch, dpc, pool, pts)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(inst)
        print("bench: multithreaded CPU baseline", file=sys.stderr, flush=True)
        rec["cpu_parallel"] = cpu_parallel(inst, out)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
