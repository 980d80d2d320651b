"""GPU parity: libdpc against the CPU oracle, element by element.

Every output is an exact integer array (Section 3's definitions with the tie
rules of the design notes), so the bar is bit-exact equality: rho, dep,
delta2 (squared, int64) and label.  Full-size workloads, too large for the
O(n^2) oracle, are checked on sampled points (the oracle's per-query
definitions) and through invariants that hold at any size.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import datagen  # noqa: E402
import oracle  # noqa: E402
import paper_2305_11335_amd as dpc  # noqa: E402

pytestmark = pytest.mark.gpu
INF = oracle.INF


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=np.int32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def gpu_run(pts, d_cut, rho_min, delta_min, skip=False):
    out = dpc.run(dev(pts), d_cut, rho_min, delta_min, skip)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def assert_same(got, want, what):
    names = ("rho", "dep", "delta2", "label")
    for name, g, w in zip(names, got, want):
        g = np.asarray(g)
        w = np.asarray(w)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            i = int(bad[0])
            raise AssertionError(f"{what}: {name} differs at {bad.size} places, first {i}: gpu {g[i]} oracle {w[i]}")


def check_invariants(pts, rho, dep, d2, lab, rho_min, delta_min, skip=False):
    """Properties that pin the outputs at any size (given rho)."""
    n = pts.shape[0]
    P = pts.astype(np.int64)
    Td = oracle.delta_threshold(delta_min)
    idx = np.arange(n, dtype=np.int64)
    key = rho.astype(np.int64) * (1 << 32) + ((1 << 32) - 1 - idx)
    assert (rho >= 1).all()
    has = dep >= 0
    assert (d2[~has] == INF).all()
    assert (key[dep[has]] > key[has]).all(), "a dependent ranks lower"
    diff = P[has] - P[dep[has]]
    assert (d2[has] == (diff * diff).sum(axis=1)).all(), "delta2 is not the squared distance"
    top = int(np.argmax(key))
    assert dep[top] == -1
    if not skip:
        assert np.flatnonzero(~has).tolist() == [top]
    noise = rho < rho_min
    assert ((lab == -1) == noise).all()
    centre = (~noise) & (d2 >= Td)
    assert (lab[centre] == idx[centre]).all()
    follow = (~noise) & (d2 < Td)
    assert (lab[follow] == lab[dep[follow]]).all()


# ---------------------------------------------------------------------------


def test_gpu_visible():
    say("device", torch.cuda.get_device_name(0))
    assert torch.cuda.is_available()
    dpc.load()


def _golden():
    import glob
    import json
    import os

    out = []
    for path in sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.json"))):
        with open(path) as f:
            g = json.load(f)
        g["delta2"] = [INF if v == "INF" else int(v) for v in g["delta2"]]
        g["name"] = os.path.basename(path)
        out.append(g)
    return out


@pytest.mark.parametrize("g", _golden(), ids=lambda g: g["name"])
def test_golden_examples(g):
    say("golden", g["name"])
    pts = np.array(g["points"], np.int32)
    got = gpu_run(pts, g["d_cut"], g["rho_min"], g["delta_min"], g["skip_noise"])
    assert_same(got, [g["rho"], g["dep"], g["delta2"], g["label"]], g["name"])


def test_random_tiny_against_oracle():
    rng = np.random.default_rng(2024)
    for case in range(250):
        n = int(rng.integers(1, 300))
        d = int(rng.integers(1, 9))
        span = int(rng.choice([2, 3, 6, 20, 200, 5000]))
        pts = datagen.random_small(case, n, d, span, offset=int(rng.integers(-100, 100)))
        d_cut = float(rng.choice([0.0, 1.0, math.sqrt(2.0), 2.5, span / 3, span * 0.1, float(span)]))
        rho_min = int(rng.integers(0, 5))
        delta_min = float(rng.choice([0.0, 1.0, 2.0, span / 4, math.inf]))
        skip = bool(rng.integers(0, 2))
        if case % 50 == 0:
            say("tiny case", case, n, d, span)
        want = oracle.run(pts, d_cut, rho_min, delta_min, skip)
        got = gpu_run(pts, d_cut, rho_min, delta_min, skip)
        assert_same(got, want, f"case {case} n={n} d={d} span={span} d_cut={d_cut}")


RAGGED = [1, 2, 31, 32, 33, 34, 39, 63, 64, 65, 97, 127, 129, 255, 257, 1000, 2047, 2049, 4095, 4096, 4097, 8193]


@pytest.mark.parametrize("n", RAGGED)
@pytest.mark.parametrize("d", [2, 3])
def test_ragged_sizes(n, d):
    say("ragged", n, d)
    pts = datagen.clustered_small(n + d, n, d, span=1 << 16, k=3, sd_frac=0.01)
    d_cut = 600.0 if d == 2 else 2000.0
    want = oracle.run(pts, d_cut, 3, 4 * d_cut)
    got = gpu_run(pts, d_cut, 3, 4 * d_cut)
    assert_same(got, want, f"n={n} d={d}")


SHAPES = [("blobs2d_10k", None), ("varden2d_1m", 20000), ("varden2d_10m", 20000), ("uniform2d_10m", 20000),
          ("mix3d_10m", 20000), ("aniso8d_10m", 12000)]


@pytest.mark.parametrize("name,n", SHAPES, ids=[s[0] for s in SHAPES])
def test_workload_shapes_against_oracle(name, n):
    inst = datagen.make(name, n=n)
    say("workload", name, inst.n, inst.d, inst.d_cut)
    want = oracle.run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min)
    got = gpu_run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min)
    assert_same(got, want, name)
    check_invariants(inst.points, *got, inst.rho_min, inst.delta_min)
    skip = gpu_run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min, skip=True)
    want_skip = oracle.run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min, True)
    assert_same(skip, want_skip, name + " skip-noise")


def test_separate_calls_match_run():
    inst = datagen.make("varden2d_1m", n=15000)
    say("separate calls", inst.n)
    P = dev(inst.points)
    rho = dpc.density(P, inst.d_cut)
    dep, d2 = dpc.dependent(P, rho)
    lab = dpc.cluster(rho, dep, d2, inst.rho_min, inst.delta_min)
    torch.cuda.synchronize()
    want = oracle.run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min)
    assert_same([t.cpu().numpy() for t in (rho, dep, d2, lab)], want, "separate calls")
    dep2, d22 = dpc.dependent(P, rho, rho_min=inst.rho_min)
    torch.cuda.synchronize()
    wd, wd2 = oracle.dependent(inst.points, want[0], inst.rho_min, True)
    assert np.array_equal(dep2.cpu().numpy(), wd) and np.array_equal(d22.cpu().numpy(), wd2)


def test_dependent_tie_hammer():
    # Densities with few distinct values make the index tie-break decide
    # almost every dependent point; small spans add distance ties.
    rng = np.random.default_rng(5)
    for case in range(60):
        n = int(rng.integers(2, 3000))
        d = int(rng.integers(1, 5))
        pts = datagen.random_small(1000 + case, n, d, int(rng.choice([4, 16, 64, 1000])))
        rho = rng.integers(-2, int(rng.integers(1, 4)), size=n).astype(np.int32)
        rho_min = int(rng.choice([0, 0, 1]))
        if case % 20 == 0:
            say("tie hammer", case, n, d)
        dep, d2 = dpc.dependent(dev(pts), dev(rho), rho_min=rho_min)
        torch.cuda.synchronize()
        wd, wd2 = oracle.dependent(pts, rho, rho_min, rho_min > 0)
        assert np.array_equal(dep.cpu().numpy(), wd), case
        assert np.array_equal(d2.cpu().numpy(), wd2), case


def test_cluster_on_given_forests():
    rng = np.random.default_rng(8)
    for case in range(40):
        n = int(rng.integers(1, 5000))
        rho = rng.integers(1, 30, size=n).astype(np.int32)
        idx = np.arange(n)
        key = rho.astype(np.int64) * (1 << 32) - idx
        order = np.argsort(-key, kind="stable")
        rank = np.empty(n, np.int64)
        rank[order] = np.arange(n)
        dep = np.full(n, -1, np.int32)
        d2 = np.full(n, INF, np.int64)
        for i in range(n):
            if rank[i] > 0:  # pick any higher-priority point
                dep[i] = order[int(rng.integers(0, rank[i]))]
                d2[i] = int(rng.integers(0, 100))
        rho_min = int(rng.integers(0, 10))
        delta_min = float(rng.choice([0.0, 3.0, 7.5, 50.0, math.inf]))
        lab = dpc.cluster(dev(rho), dev(dep), dev(d2, np.int64), rho_min, delta_min)
        torch.cuda.synchronize()
        want = oracle.cluster(rho, dep, d2, rho_min, oracle.delta_threshold(delta_min))
        assert np.array_equal(lab.cpu().numpy(), want), case


def test_cluster_rejects_non_forest():
    say("not a forest")
    rho = np.array([2, 2, 2], np.int32)
    d2 = np.array([1, 1, 1], np.int64)
    for dep in ([1, 2, 0], [-1, 2, 0], [-1, 7, 0], [-1, 0, -1]):
        with pytest.raises(dpc.DPCError) as e:
            dpc.cluster(dev(rho), dev(np.array(dep, np.int32)), dev(d2, np.int64), 0, 5.0)
        assert e.value.status == 3


@pytest.mark.parametrize("d,span", [(1, 3_000_000_000), (2, 1 << 30), (3, 1 << 29), (8, 1 << 28)])
def test_wide_coordinates_int64_path(d, span):
    say("int64 path", d, span)
    rng = np.random.default_rng(d)
    lo = -(1 << 31) + 5
    n = 3000
    centres = rng.integers(lo, lo + span, size=(4, d))
    pts = centres[rng.integers(0, 4, size=n)] + rng.integers(-200_000, 200_000, size=(n, d))
    pts = np.clip(pts, lo, lo + span - 1).astype(np.int32)
    pts[0] = lo
    pts[1] = lo + span - 1
    want = oracle.run(pts, 150_000.0, 2, 1e6)
    got = gpu_run(pts, 150_000.0, 2, 1e6)
    assert_same(got, want, f"int64 d={d}")


def test_range_error():
    pts = np.array([[-(2 ** 31)] * 8, [2 ** 31 - 1] * 8], np.int32)
    with pytest.raises(dpc.DPCError) as e:
        gpu_run(pts, 1.0, 0, 1.0)
    assert e.value.status == 2
    w = 3037000499
    ok = np.array([[-1518500249], [-1518500249 + w]], np.int32)
    got = gpu_run(ok, 1.0, 0, 1.0)
    assert got[2].tolist() == [INF, w * w]


def test_closed_forms_on_device():
    pts = datagen.random_small(77, 3000, 2, 40)
    rho, dep, d2, lab = gpu_run(pts, 0.0, 1, 1.0)
    _, inv, counts = np.unique(pts, axis=0, return_inverse=True, return_counts=True)
    assert np.array_equal(rho, counts[inv.reshape(-1)])
    rho, dep, d2, lab = gpu_run(pts, math.inf, 1, 1.0)
    assert (rho == 3000).all()
    want = oracle.run(pts, math.inf, 1, 1.0)
    assert_same([rho, dep, d2, lab], want, "d_cut = inf")


def test_deterministic_across_runs_and_streams():
    inst = datagen.make("varden2d_1m", n=200_000)
    say("determinism", inst.n)
    P = dev(inst.points)
    a = [t.cpu() for t in dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, stream=s)
    s.synchronize()
    c = [t.cpu() for t in dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min)]
    for x, y, z in zip(a, b, c):
        assert torch.equal(x, y.cpu()) and torch.equal(x, z)


def oracle_at(points, T, rho, q):
    """The oracle's per-query density and dependent point (Section 3,
    Definitions 1-3) for the queries q, split over the host threads (each
    call is a plain O(n) scan per query; ctypes releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import cpu_baseline

    workers = max(1, min(16, cpu_baseline.threads_available()))
    chunks = [c for c in np.array_split(np.asarray(q, np.int64), workers) if c.size]
    with ThreadPoolExecutor(workers) as ex:
        dens = list(ex.map(lambda c: oracle.density_at(points, T, c), chunks))
        deps = list(ex.map(lambda c: oracle.dependent_at(points, rho, c), chunks))
    return (np.concatenate(dens), np.concatenate([a for a, _ in deps]), np.concatenate([b for _, b in deps]))


def full_size_samples(rho, dep, d2, n, count=1000, seed=99):
    """count random points plus the points whose searches are longest: the
    densest point, every root, the points with the largest finite delta2
    (density peaks) and the least dense points."""
    rng = np.random.default_rng(seed)
    q = rng.choice(n, size=count, replace=False)
    finite = np.flatnonzero(dep >= 0)
    peaks = finite[np.argsort(d2[finite])[-32:]]
    sparse = np.argsort(rho, kind="stable")[:16]
    extra = np.concatenate([[int(np.argmax(rho))], np.flatnonzero(dep < 0)[:8], peaks, sparse])
    return np.unique(np.concatenate([q, extra])).astype(np.int64)


FULL_SIZE = ["varden2d_1m", "varden2d_10m", "uniform2d_10m", "mix3d_10m",
             pytest.param("aniso8d_10m", marks=pytest.mark.timeout(900))]


@pytest.mark.parametrize("name", FULL_SIZE)
def test_full_size_exact(name):
    """The whole output arrays at full size, in the launch configuration
    bench.py times: bit-equal to the independently written multithreaded CPU
    k-d tree version (itself checked against the oracle on the CPU), at least
    1000 sampled points bit-equal to the oracle's per-query definitions, and
    the invariants that pin every output given rho."""
    import cpu_baseline

    inst = datagen.make(name)
    say("full size", name, inst.n, inst.d, inst.d_cut)
    rho, dep, d2, lab = gpu_run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min)
    say("  cpu k-d tree version, threads", cpu_baseline.threads_available())
    want = cpu_baseline.run(inst.points, inst.d_cut, inst.rho_min, inst.delta_min)
    assert_same([rho, dep, d2, lab], want, f"{name} against the CPU version")
    q = full_size_samples(rho, dep, d2, inst.n)
    say("  oracle samples", q.size)
    T = oracle.square_threshold(inst.d_cut)
    w_rho, w_dep, w_d2 = oracle_at(inst.points, T, rho, q)
    assert np.array_equal(rho[q], w_rho), "sampled density"
    assert np.array_equal(dep[q], w_dep) and np.array_equal(d2[q], w_d2), "sampled dependent"
    check_invariants(inst.points, rho, dep, d2, lab, inst.rho_min, inst.delta_min)


def test_measurement_flags_leave_outputs_unchanged():
    inst = datagen.make("varden2d_1m", n=100_000)
    say("measurement flags", inst.n)
    P = dev(inst.points)
    plain = [t.cpu() for t in dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min)]
    timed = [t.cpu() for t in dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, time_stages=True)]
    st = dpc.last_stats()
    assert all(st["stage_ms"][k] > 0 for k in dpc.STAGES)
    counted = [t.cpu() for t in dpc.run(P, inst.d_cut, inst.rho_min, inst.delta_min, count_work=True)]
    wk = dpc.last_stats()
    for a, b, c in zip(plain, timed, counted):
        assert torch.equal(a, b) and torch.equal(a, c)
    rho = plain[0].numpy().astype(np.int64)
    # every counted point is either inside a contained node or was tested
    assert wk["density_contained"] <= int(rho.sum()) <= wk["density_contained"] + wk["density_pairs"]
    assert wk["dependent_pairs"] >= inst.n - 1 and wk["density_nodes"] > 0 and wk["dependent_nodes"] > 0
