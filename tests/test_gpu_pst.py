"""The priority-search k-d tree backend: the tree of Section 4.2 with one
point stored per node, searched by the priority nearest-neighbour query of
Algorithm 1.

Its outputs must equal the oracle's on small inputs and the default k-d
tree's bit for bit everywhere.  Sizes straddle powers of two (the last level
of the heap-shaped tree is then empty, full or partly filled) and the tree
heights where the per-node reductions change form (subtrees of 64 and 4096
points).
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
def test_sizes_around_powers_of_two(d):
    for n in (1, 2, 3, 4, 7, 8, 9, 63, 64, 65, 127, 128, 1023, 1025, 4095, 4097, 8191, 9000):
        pts = datagen.clustered_small(n * 11 + d, n, d, span=1 << 15, k=4, sd_frac=0.02)
        d_cut = {1: 30.0, 2: 300.0, 3: 900.0, 5: 2500.0, 8: 5000.0}[d]
        got = host(dpc.run(dev(pts), d_cut, 2, 3 * d_cut, pst=True))
        same(got, oracle.run(pts, d_cut, 2, 3 * d_cut), f"d={d} n={n}")
    say("d", d, "ok")


def test_random_small_cases():
    rng = np.random.default_rng(4202)
    for case in range(60):
        n = int(rng.integers(1, 3000))
        d = int(rng.integers(1, 9))
        span = int(rng.choice([3, 20, 300, 5000]))  # small spans: many ties and duplicates
        pts = datagen.random_small(case + 900, n, d, span)
        d_cut = float(rng.choice([0.0, 1.5, span / 3, float(span)]))
        rho_min = int(rng.integers(0, 4))
        delta_min = float(rng.choice([0.0, 2.0, span / 4, math.inf]))
        skip = bool(rng.integers(0, 2))
        got = host(dpc.run(dev(pts), d_cut, rho_min, delta_min, skip, pst=True))
        same(got, oracle.run(pts, d_cut, rho_min, delta_min, skip), f"case {case} n={n} d={d} skip={skip}")


def test_wide_coordinates():
    # spans near 2^29 (squared distances beyond 2^53), and in one dimension a
    # span of 3e9, just inside the int64 range check (9e18 < 2^63)
    for d in (2, 3):
        pts = datagen.random_small(177 + d, 5000, d, span=1 << 29, offset=-(1 << 28))
        got = host(dpc.run(dev(pts), float(1 << 25), 1, float(1 << 27), pst=True))
        same(got, oracle.run(pts, float(1 << 25), 1, float(1 << 27)), f"wide d={d}")
    line = np.array([[-1_500_000_000], [1_500_000_000], [0], [5], [-7], [1_000_000_000]], np.int32)
    same(host(dpc.run(dev(line), 3.0, 1, 10.0, pst=True)), oracle.run(line, 3.0, 1, 10.0), "int32 range")


@pytest.mark.parametrize("name,n", [("varden2d_10m", 300_000), ("mix3d_10m", 200_000), ("aniso8d_10m", 40_000)])
def test_equals_default_tree(name, n):
    x = datagen.make(name, n=n)
    P = dev(x.points)
    for skip in (False, True):
        want = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min, skip))
        got = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min, skip, pst=True))
        same(got, want, f"{name} n={n} skip={skip}")
    say(name, "ok")


def test_full_size_2d():
    x = datagen.make("varden2d_10m")
    P = dev(x.points)
    want = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
    got = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min, pst=True))
    say("priority-search tree done")
    same(got, want, "varden2d_10m full size")


def test_backend_setting_and_autotuner_keep_outputs():
    x = datagen.make("varden2d_1m", n=150_000)
    P = dev(x.points)
    before = dpc.dependent_backend(2)
    try:
        ref = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
        dpc.set_dependent_backend(2, "priority_search_tree")
        same(host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min)), ref, "priority-search tree by setting")
        r = dpc.autotune_dependent(P, x.d_cut, x.rho_min, x.delta_min)
        say("autotune_dependent", r)
        assert set(r["ms"]) == set(dpc.BACKENDS) and all(t > 0 for t in r["ms"].values())
        assert r["chosen"] == min(r["ms"], key=r["ms"].get) and dpc.dependent_backend(2) == r["chosen"]
        same(host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min)), ref, "after the backend autotuner")
    finally:
        dpc.set_dependent_backend(2, before)


def test_degenerate_inputs():
    # every point the same, equally spaced collinear points (a distance tie at
    # every step), and a cluster with one far point
    cases = [np.zeros((n, 2), np.int32) for n in (1, 1500, 5000)]
    cases.append(np.stack([np.arange(3000) * 7, np.zeros(3000)], 1).astype(np.int32))
    blob = datagen.clustered_small(93, 4000, 3, span=1 << 12, k=1, sd_frac=0.05)
    blob[17] = [1 << 28, 1 << 28, 1 << 28]
    cases.append(blob)
    for k, pts in enumerate(cases):
        for d_cut, rho_min, delta_min in ((0.0, 1, 1.0), (10.0, 2, 30.0)):
            got = host(dpc.run(dev(pts), d_cut, rho_min, delta_min, pst=True))
            same(got, oracle.run(pts, d_cut, rho_min, delta_min), f"case {k} n={pts.shape[0]} d_cut={d_cut}")
