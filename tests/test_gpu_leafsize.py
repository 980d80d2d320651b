"""GPU parity under every k-d tree leaf size (16, 32 and 64 points).

The leaf size is a tuning choice: every output must be the same with any,
equal to the oracle on small inputs and equal between the sizes on the
full-size workloads.  The autotuner must pick one of them and leave the
outputs unchanged.
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


@pytest.fixture(params=[16, 32, 64], ids=["leaf16", "leaf32", "leaf64"])
def leaf(request):
    before = {d: dpc.leaf_size(d) for d in range(1, 9)}
    for d in range(1, 9):
        dpc.set_leaf_size(d, request.param)
    yield request.param
    for d, s in before.items():
        dpc.set_leaf_size(d, s)


def test_random_tiny(leaf):
    rng = np.random.default_rng(300 + leaf)
    for case in range(120):
        n = int(rng.integers(1, 400))
        d = int(rng.integers(1, 9))
        span = int(rng.choice([3, 20, 300, 5000]))
        pts = datagen.random_small(case + 7 * leaf, n, d, span)
        d_cut = float(rng.choice([0.0, 1.5, span / 3, float(span)]))
        rho_min = int(rng.integers(0, 4))
        delta_min = float(rng.choice([0.0, 2.0, span / 4, math.inf]))
        skip = bool(rng.integers(0, 2))
        got = host(dpc.run(dev(pts), d_cut, rho_min, delta_min, skip))
        same(got, oracle.run(pts, d_cut, rho_min, delta_min, skip), f"leaf {leaf} case {case} n={n} d={d}")


@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_ragged_sizes(leaf, d):
    for n in (1, 15, 16, 17, 31, 33, 63, 64, 65, 127, 129, 513, 1023, 1025, 2047, 2049, 4097):
        pts = datagen.clustered_small(n * 3 + d, n, d, span=1 << 16, k=3, sd_frac=0.01)
        d_cut = {2: 600.0, 3: 2000.0, 5: 6000.0, 8: 12000.0}[d]
        got = host(dpc.run(dev(pts), d_cut, 3, 4 * d_cut))
        same(got, oracle.run(pts, d_cut, 3, 4 * d_cut), f"leaf {leaf} n={n} d={d}")


@pytest.mark.parametrize("name,n", [("varden2d_10m", 15000), ("mix3d_10m", 15000), ("aniso8d_10m", 8000)])
def test_workload_shapes(leaf, name, n):
    x = datagen.make(name, n=n)
    got = host(dpc.run(dev(x.points), x.d_cut, x.rho_min, x.delta_min))
    same(got, oracle.run(x.points, x.d_cut, x.rho_min, x.delta_min), f"leaf {leaf} {name}")


def test_batch(leaf):
    probs = [(x.points, x.d_cut, x.rho_min, x.delta_min)
             for x in datagen.batch_instances(seed=17, count=24, n_hi=6000)]
    outs, st = dpc.batch_run([(dev(p), dc, rm, dm) for p, dc, rm, dm in probs], check=False)
    assert st == [0] * len(probs)
    for k, (p, dc, rm, dm) in enumerate(probs):
        same(host(outs[k]), oracle.run(p, dc, rm, dm), f"leaf {leaf} batch instance {k} d={p.shape[1]}")


@pytest.mark.parametrize("name", ["varden2d_10m", "mix3d_10m"])
def test_full_size_leaf_sizes_agree(name):
    x = datagen.make(name)
    P = dev(x.points)
    before = dpc.leaf_size(x.d)
    try:
        res = {}
        for size in (16, 32, 64):
            dpc.set_leaf_size(x.d, size)
            res[size] = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
            say(name, "leaf", size, "done")
    finally:
        dpc.set_leaf_size(x.d, before)
    same(res[16], res[64], f"{name}: leaf 16 against leaf 64")
    same(res[32], res[64], f"{name}: leaf 32 against leaf 64")


def test_autotune_keeps_outputs():
    x = datagen.make("mix3d_10m", n=300_000)
    P = dev(x.points)
    before = dpc.leaf_size(3)
    try:
        ref = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
        r = dpc.autotune(P, x.d_cut, x.rho_min, x.delta_min)
        say("autotune", r)
        assert r["chosen"] in dpc.LEAF_SIZES and dpc.leaf_size(3) == r["chosen"]
        assert all(r["ms"][size] > 0 for size in dpc.LEAF_SIZES)
        assert r["chosen"] == min(dpc.LEAF_SIZES, key=lambda size: r["ms"][size])
        same(host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min)), ref, "after autotune")
    finally:
        dpc.set_leaf_size(3, before)
