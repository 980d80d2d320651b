"""The Fenwick-tree dependent-point backend (Section 5, Algorithm 2).

Its outputs must equal the oracle's on small inputs and the priority-search
k-d tree's bit for bit everywhere: below 1024 points every range is scanned
directly; above, the k-d tree ranges take part, so the sizes straddle 1024,
2048, 4096 and reach several tree levels, with ragged tails.
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def host(out):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def same(got, want, what):
    for name, g, w in zip(("rho", "dep", "delta2", "label"), got, want):
        g, w = np.asarray(g), np.asarray(w)
        if not np.array_equal(g, w):
            i = int(np.flatnonzero(g != w)[0])
            raise AssertionError(f"{what}: {name} differs at {int((g != w).sum())} places, first {i}: {g[i]} vs {w[i]}")


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
def test_sizes_around_the_scan_limit(d):
    for n in (1, 2, 63, 1023, 1024, 1025, 2047, 2048, 2049, 3071, 4097, 9000):
        pts = datagen.clustered_small(n * 7 + d, n, d, span=1 << 15, k=4, sd_frac=0.02)
        d_cut = {1: 30.0, 2: 300.0, 3: 900.0, 5: 2500.0, 8: 5000.0}[d]
        got = host(dpc.run(dev(pts), d_cut, 2, 3 * d_cut, fenwick=True))
        same(got, oracle.run(pts, d_cut, 2, 3 * d_cut), f"d={d} n={n}")
    say("d", d, "ok")


def test_random_small_cases():
    rng = np.random.default_rng(2305)
    for case in range(60):
        n = int(rng.integers(1, 3000))
        d = int(rng.integers(1, 9))
        span = int(rng.choice([3, 20, 300, 5000]))  # small spans: many ties and duplicates
        pts = datagen.random_small(case + 500, n, d, span)
        d_cut = float(rng.choice([0.0, 1.5, span / 3, float(span)]))
        rho_min = int(rng.integers(0, 4))
        delta_min = float(rng.choice([0.0, 2.0, span / 4, math.inf]))
        skip = bool(rng.integers(0, 2))
        got = host(dpc.run(dev(pts), d_cut, rho_min, delta_min, skip, fenwick=True))
        same(got, oracle.run(pts, d_cut, rho_min, delta_min, skip), f"case {case} n={n} d={d} skip={skip}")


def test_wide_coordinates_take_the_integer_path():
    # spans near 2^29: squared distances beyond 2^53, exact int64 arithmetic
    for d in (2, 3):
        pts = datagen.random_small(77 + d, 5000, d, span=1 << 29, offset=-(1 << 28))
        got = host(dpc.run(dev(pts), float(1 << 25), 1, float(1 << 27), fenwick=True))
        same(got, oracle.run(pts, float(1 << 25), 1, float(1 << 27)), f"wide d={d}")


@pytest.mark.parametrize("name,n", [("varden2d_10m", 200_000), ("mix3d_10m", 150_000), ("aniso8d_10m", 40_000)])
def test_equals_priority_search_tree(name, n):
    x = datagen.make(name, n=n)
    P = dev(x.points)
    for skip in (False, True):
        want = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min, skip))
        got = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min, skip, fenwick=True))
        same(got, want, f"{name} n={n} skip={skip}")
    say(name, "ok")


def test_full_size_2d():
    x = datagen.make("varden2d_10m")
    P = dev(x.points)
    want = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
    say("tree done")
    got = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min, fenwick=True))
    say("fenwick done")
    same(got, want, "varden2d_10m full size")


def test_backend_setting_and_autotuner_keep_outputs():
    x = datagen.make("mix3d_10m", n=200_000)
    P = dev(x.points)
    before = dpc.dependent_backend(3)
    try:
        ref = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
        dpc.set_dependent_backend(3, "fenwick")
        same(host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min)), ref, "Fenwick backend by setting")
        r = dpc.autotune_dependent(P, x.d_cut, x.rho_min, x.delta_min)
        say("autotune_dependent", r)
        assert r["chosen"] in dpc.BACKENDS and dpc.dependent_backend(3) == r["chosen"]
        assert r["ms"]["priority_tree"] > 0 and r["ms"]["fenwick"] > 0
        assert r["chosen"] == min(r["ms"], key=r["ms"].get)
        same(host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min)), ref, "after the backend autotuner")
    finally:
        dpc.set_dependent_backend(3, before)


def test_degenerate_inputs():
    # every point the same (all distances 0, all densities n), equally spaced
    # collinear points (a distance tie at every step), and a cluster with one
    # far point; sizes reach the k-d tree ranges
    cases = [np.zeros((n, 2), np.int32) for n in (1500, 5000)]
    cases.append(np.stack([np.arange(3000) * 7, np.zeros(3000)], 1).astype(np.int32))
    blob = datagen.clustered_small(91, 4000, 3, span=1 << 12, k=1, sd_frac=0.05)
    blob[17] = [1 << 28, 1 << 28, 1 << 28]
    cases.append(blob)
    for k, pts in enumerate(cases):
        for d_cut, rho_min, delta_min in ((0.0, 1, 1.0), (10.0, 2, 30.0)):
            got = host(dpc.run(dev(pts), d_cut, rho_min, delta_min, fenwick=True))
            same(got, oracle.run(pts, d_cut, rho_min, delta_min), f"case {k} n={pts.shape[0]} d_cut={d_cut}")
