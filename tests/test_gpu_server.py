"""GPU tests of the served path (dpc_server_*).

A request's outputs must be bit-identical to dpc_run's on the same arguments
whatever it was batched with; admission must keep the summed workspace
bounds of the requests in flight within the budget, and the batches'
workspaces within their bounds.  The workspace bound itself is checked
against the workspace that dpc_run reports.
"""
import sys
import threading
import time

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


def same(got, want, what):
    for name, g, w in zip(("rho", "dep", "delta2", "label"), got, want):
        g, w = g.cpu().numpy(), w.cpu().numpy() if hasattr(w, "cpu") else np.asarray(w)
        if not np.array_equal(g, w):
            i = int(np.flatnonzero(g != w)[0])
            raise AssertionError(f"{what}: {name} differs at {int((g != w).sum())} places, first {i}: {g[i]} vs {w[i]}")


def pool(count=24, n_hi=120_000, seed=21):
    return datagen.served_instances(seed=seed, count=count, n_hi=n_hi)


def test_workspace_bound_covers_dpc_run():
    for name, n, d in (("blobs2d_10k", 10_000, 2), ("varden2d_1m", 300_000, 2), ("mix3d_10m", 200_000, 3),
                       ("aniso8d_10m", 50_000, 8)):
        inst = datagen.make(name, n=n)
        dpc.run(dev(inst.points), inst.d_cut, inst.rho_min, inst.delta_min, time_stages=True)
        used = dpc.last_stats()["workspace_bytes"]
        bound = dpc.workspace_bytes(n, d)
        say(name, n, d, "workspace", used, "bound", bound)
        assert 0 < used <= bound
        assert bound < 1.6 * used  # the bound is not loose either
    for n, d in ((1, 1), (33, 5), (2049, 3), (5000, 8)):
        p = datagen.random_small(n + d, n, d, 1 << 16)
        dpc.run(dev(p), 500.0, 2, 1000.0, time_stages=True)
        assert 0 < dpc.last_stats()["workspace_bytes"] <= dpc.workspace_bytes(n, d)


def test_served_equals_alone_under_concurrent_arrivals():
    reqs = pool()
    pts = [dev(x.points) for x in reqs]
    order = np.random.default_rng(3).permutation(np.repeat(np.arange(len(reqs)), 2))
    say("requests", len(order), "pool points", sum(x.n for x in reqs))
    done = []
    with dpc.Server(hbm_budget_bytes=8 << 30, slots=3, max_batch=16) as srv:
        tickets = []

        def submitter():
            rng = np.random.default_rng(4)
            for k in order:
                x = reqs[k]
                t, res = srv.submit(pts[k], x.d_cut, x.rho_min, x.delta_min, skip_noise=bool(k % 3 == 0))
                tickets.append((t, k, res))
                time.sleep(float(rng.exponential(0.002)))

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for t, k, res in tickets:
            info = srv.wait(t)
            assert info["done"] == 1 and info["status"] == 0
            assert info["submit_ns"] <= info["admit_ns"] <= info["done_ns"]
            done.append((k, res, info))
        st = srv.stats()
    say("server stats", st)
    assert st["submitted"] == st["completed"] == len(order)
    assert st["over_footprint"] == 0 and st["max_admitted_bytes"] <= 8 << 30
    assert st["max_workspace_bytes"] > 0
    for k, res, info in done:
        x = reqs[k]
        alone = dpc.run(pts[k], x.d_cut, x.rho_min, x.delta_min, skip_noise=bool(k % 3 == 0))
        torch.cuda.synchronize()
        same(res, alone, f"request of pool entry {k} (batch of {info['batch_size']})")


def test_batching_and_budget():
    reqs = pool(count=16, n_hi=60_000, seed=22)
    pts = [dev(x.points) for x in reqs]
    # footprint: workspace bound plus the request's points and outputs
    fps = [dpc.workspace_bytes(x.n, x.d) + x.n * (4 * x.d + 20) for x in reqs]
    # one slot and a queue filled at once: later requests are batched together
    with dpc.Server(hbm_budget_bytes=64 << 30, slots=1, max_batch=64) as srv:
        tk = [srv.submit(p, x.d_cut, x.rho_min, x.delta_min) for p, x in zip(pts, reqs)]
        infos = [srv.wait(t) for t, _ in tk]
        st = srv.stats()
    assert all(i["status"] == 0 for i in infos)
    assert [i["footprint"] for i in infos] == fps
    assert st["batches"] < len(reqs) and st["max_batch_seen"] > 1
    for (t, res), x, p in zip(tk, reqs, pts):
        same(res, dpc.run(p, x.d_cut, x.rho_min, x.delta_min), "batched request")
    # a budget that holds the two largest requests at most: never more in flight
    budget = sorted(fps)[-1] + sorted(fps)[-2]
    with dpc.Server(hbm_budget_bytes=budget, slots=4, max_batch=8) as srv:
        tk = [srv.submit(p, x.d_cut, x.rho_min, x.delta_min) for p, x in zip(pts, reqs)]
        infos = [srv.wait(t) for t, _ in tk]
        st = srv.stats()
    say("small budget", budget, st)
    assert all(i["status"] == 0 for i in infos)
    assert st["max_admitted_bytes"] <= budget and st["over_footprint"] == 0
    for (t, res), x, p in zip(tk, reqs, pts):
        same(res, dpc.run(p, x.d_cut, x.rho_min, x.delta_min), "request under a small budget")
    # a request larger than the whole budget is refused at submission
    with dpc.Server(hbm_budget_bytes=min(fps) // 2, slots=1, max_batch=1) as srv:
        with pytest.raises(dpc.DPCError) as e:
            srv.submit(pts[0], reqs[0].d_cut, reqs[0].rho_min, reqs[0].delta_min)
        assert e.value.status == dpc._binding.ERR_OOM
        assert srv.stats()["rejected"] == 1


def test_failing_request_in_the_mix():
    ok = datagen.clustered_small(31, 4000, 3, span=1 << 16)
    wide = np.array([[0, 0, 0], [2**31 - 1, 2**31 - 1, 2**31 - 1], [-2**31, -2**31, -2**31]], np.int32)
    with dpc.Server(hbm_budget_bytes=1 << 30, slots=1, max_batch=8) as srv:
        a, ra = srv.submit(dev(ok), 2500.0, 3, 1e4)
        b, _ = srv.submit(dev(wide), 1.0, 0, 1.0)
        c, rc = srv.submit(dev(ok[:1500]), 2500.0, 3, 1e4)
        ia, ib, ic = srv.wait(a), srv.wait(b), srv.wait(c)
        with pytest.raises(dpc.DPCError):
            srv.poll(a)  # forgotten once reported
    assert (ia["status"], ib["status"], ic["status"]) == (0, dpc._binding.ERR_RANGE, 0)
    same(ra, oracle.run(ok, 2500.0, 3, 1e4), "request beside a failing one")
    same(rc, oracle.run(ok[:1500], 2500.0, 3, 1e4), "request beside a failing one")


def test_poll_until_done_and_destroy_drains():
    reqs = pool(count=6, n_hi=30_000, seed=23)
    pts = [dev(x.points) for x in reqs]
    srv = dpc.Server(hbm_budget_bytes=1 << 30, slots=2, max_batch=4)
    tk = [srv.submit(p, x.d_cut, x.rho_min, x.delta_min) for p, x in zip(pts, reqs)]
    t0, res0 = tk[0]
    deadline = time.time() + 60
    while True:
        info = srv.poll(t0)
        if info["done"]:
            break
        assert time.time() < deadline
        time.sleep(0.001)
    assert info["status"] == 0
    srv.close()  # the other requests run to completion first
    for (t, res), x, p in zip(tk, reqs, pts):
        same(res, dpc.run(p, x.d_cut, x.rho_min, x.delta_min), "request finished at destroy")
