"""Plans: one dpc_run recorded and replayed, eagerly or as a HIP graph.

Every replay must give exactly what dpc_run gives on the points' current
contents (equal to the oracle on small inputs), as long as the points stay
inside the bounds the plan was made for; outside them the replay's status
word reads the range error, and the plan works again once the points are
back inside.  Graph replays are checked one by one with eager work between
them.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import datagen  # noqa: E402
import oracle  # noqa: E402
import paper_2305_11335_amd as dpc  # noqa: E402
from paper_2305_11335_amd import _binding  # noqa: E402

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


def within(pts, ref, seed):
    """A new draw of the same shape, clipped into the per-axis bounds of ref."""
    rng = np.random.default_rng(seed)
    lo, hi = ref.min(axis=0), ref.max(axis=0)
    new = ref[rng.permutation(ref.shape[0])] + rng.integers(-40, 41, size=ref.shape)
    return np.clip(new, lo, hi).astype(np.int32)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("n", [1, 17, 700, 4097])
def test_first_run_and_replays_match_oracle(d, n):
    pts = datagen.clustered_small(n * 11 + d, n, d, span=1 << 14, k=3, sd_frac=0.02)
    d_cut = {1: 40.0, 2: 300.0, 3: 900.0, 5: 2500.0, 8: 5000.0}[d]
    P = dev(pts)
    with dpc.Plan(P, d_cut, 2, 3 * d_cut) as plan:
        same(host(plan.out), oracle.run(pts, d_cut, 2, 3 * d_cut), f"created d={d} n={n}")
        for rep in range(2):
            new = within(pts, pts, 100 * rep + n + d)
            P.copy_(dev(new))
            plan.launch()
            assert plan.status() == 0
            same(host(plan.out), oracle.run(new, d_cut, 2, 3 * d_cut), f"replay {rep} d={d} n={n}")


def test_skip_noise_and_empty():
    pts = datagen.clustered_small(5, 3000, 3, span=1 << 15, k=4, sd_frac=0.01)
    P = dev(pts)
    with dpc.Plan(P, 500.0, 5, 2000.0, skip_noise=True) as plan:
        plan.launch()
        same(host(plan.out), oracle.run(pts, 500.0, 5, 2000.0, True), "skip noise")
    E = torch.empty((0, 4), dtype=torch.int32, device="cuda")
    with dpc.Plan(E, 10.0, 1, 10.0) as plan:
        plan.launch()
        plan.capture()
        plan.launch()
        assert plan.status() == 0
        assert all(t.numel() == 0 for t in plan.out)


@pytest.mark.parametrize("name", ["varden2d_10m", "mix3d_10m"])
def test_full_size_replays(name):
    x = datagen.make(name)
    P = dev(x.points)
    want = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
    with dpc.Plan(P, x.d_cut, x.rho_min, x.delta_min) as plan:
        same(host(plan.out), want, f"{name} created")
        say(name, "created")
        for t in plan.out:
            t.fill_(-7)
        plan.launch()
        same(host(plan.out), want, f"{name} replay")
        say(name, "replayed")
        new = within(x.points, x.points, 5)
        P.copy_(dev(new))
        plan.launch()
        assert plan.status() == 0
        same(host(plan.out), host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min)), f"{name} replay on new points")
        say(name, "replayed on new points")


def test_graph_replays_with_eager_work_between():
    x = datagen.make("varden2d_10m", n=400_000)
    P = dev(x.points)
    s = torch.cuda.Stream()
    with dpc.Plan(P, x.d_cut, x.rho_min, x.delta_min) as plan:
        plan.capture(s)
        for rep in range(4):
            new = within(x.points, x.points, 50 + rep)
            P.copy_(dev(new))
            for t in plan.out:
                t.fill_(-3)
            # eager work of the program's own between the replays
            ref = host(dpc.run(P, x.d_cut, x.rho_min, x.delta_min))
            torch.cuda.synchronize()
            plan.launch(s)
            assert plan.status(s) == 0
            s.synchronize()
            same(host(plan.out), ref, f"graph replay {rep}")
            say("graph replay", rep, "ok")


def test_graph_replays_small_match_oracle():
    pts = datagen.clustered_small(77, 5000, 4, span=1 << 16, k=5, sd_frac=0.01)
    P = dev(pts)
    s = torch.cuda.Stream()
    with dpc.Plan(P, 1500.0, 3, 6000.0, stream=s) as plan:
        plan.capture(s)
        for rep in range(3):
            new = within(pts, pts, 900 + rep)
            P.copy_(dev(new))
            torch.cuda.synchronize()
            plan.launch(s)
            s.synchronize()
            same(host(plan.out), oracle.run(new, 1500.0, 3, 6000.0), f"small graph replay {rep}")


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_points_outside_the_plan_report_range(graph):
    pts = datagen.clustered_small(31, 6000, 3, span=1 << 15, k=3, sd_frac=0.02)
    P = dev(pts)
    s = torch.cuda.Stream()
    with dpc.Plan(P, 700.0, 2, 2800.0, stream=s) as plan:
        if graph:
            plan.capture(s)
        hi = pts.max(axis=0)
        lo = pts.min(axis=0)
        for k, bad in enumerate(([hi[0] + 1, lo[1], lo[2]], [lo[0], lo[1] - 1000, lo[2]],
                                 [hi[0] + (1 << 20), hi[1] + (1 << 20), lo[2] - (1 << 20)])):
            moved = pts.copy()
            moved[123 + k] = bad
            P.copy_(dev(moved))
            torch.cuda.synchronize()
            plan.launch(s)
            assert plan.status(s) == _binding.ERR_RANGE, f"case {k}"
            # back inside: the plan is exact again
            P.copy_(dev(pts))
            torch.cuda.synchronize()
            plan.launch(s)
            assert plan.status(s) == 0
            same(host(plan.out), oracle.run(pts, 700.0, 2, 2800.0), f"after range case {k}")


def test_plan_creation_errors_match_dpc_run():
    P = dev(np.array([[-(2**31), 0], [2**31 - 1, 0], [0, 5]], dtype=np.int64))
    with pytest.raises(dpc.DPCError) as e:
        dpc.Plan(P, 1.0, 1, 1.0)
    assert e.value.status == _binding.ERR_RANGE


def test_batch_plan_replays_match_batch_run():
    insts = datagen.batch_instances(seed=21, count=24, n_hi=8000)
    probs = [(x.points, x.d_cut, x.rho_min, x.delta_min) for x in insts]
    P = [dev(p) for p, *_ in probs]

    def batch_now():
        outs, st = dpc.batch_run([(t, dc, rm, dm) for t, (_, dc, rm, dm) in zip(P, probs)], check=False)
        assert st == [0] * len(probs)
        return [host(o) for o in outs]

    want = batch_now()
    s = torch.cuda.Stream()
    with dpc.BatchPlan([(t, dc, rm, dm) for t, (_, dc, rm, dm) in zip(P, probs)], stream=s) as plan:
        assert plan.statuses() == [0] * len(probs)
        for k in range(len(probs)):
            same(host(plan.results[k]), want[k], f"created, instance {k}")
        for rep in range(3):
            news = [within(p, p, 300 + 17 * rep + i) for i, (p, *_) in enumerate(probs)]
            for t, a in zip(P, news):
                t.copy_(dev(a))
            torch.cuda.synchronize()
            if rep == 1:
                plan.capture(s)
            plan.launch(s)
            assert plan.status(s) == 0
            s.synchronize()
            ref = batch_now()
            for k in range(len(probs)):
                same(host(plan.results[k]), ref[k], f"replay {rep}, instance {k}")
            say("batch plan replay", rep, "ok")
        # one instance's point leaves its planned bounds: the range status,
        # then exact results again once it is back
        moved = news[3].copy()
        moved[0] = news[3].max(axis=0) + 5
        P[3].copy_(dev(moved))
        torch.cuda.synchronize()
        plan.launch(s)
        assert plan.status(s) == _binding.ERR_RANGE
        P[3].copy_(dev(news[3]))
        torch.cuda.synchronize()
        plan.launch(s)
        assert plan.status(s) == 0
        s.synchronize()
        ref = batch_now()
        for k in range(len(probs)):
            same(host(plan.results[k]), ref[k], f"after the range case, instance {k}")


def test_batch_plan_refuses_a_failing_instance():
    good = datagen.clustered_small(5, 3000, 2, span=1 << 16)
    wide = np.array([[0, 0], [2**31 - 1, 2**31 - 1], [-2**31, -2**31]], np.int32)
    with pytest.raises(dpc.DPCError) as e:
        dpc.BatchPlan([(dev(good), 700.0, 3, 2800.0), (dev(wide), 1.0, 0, 1.0)])
    assert e.value.status == _binding.ERR_RANGE
