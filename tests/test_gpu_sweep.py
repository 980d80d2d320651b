"""GPU parity of the parameter sweeps (dpc_density_sweep, dpc_cluster_sweep).

Row k of a sweep must equal the single call with parameter k, bit for bit,
and the oracle on small inputs.
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


@pytest.mark.parametrize("name,n", [("varden2d_1m", 200_000), ("mix3d_10m", 60_000), ("aniso8d_10m", 20_000)])
def test_density_sweep_rows_equal_single_calls(name, n):
    inst = datagen.make(name, n=n)
    P = dev(inst.points)
    # zero, small, the workload's own, large (beyond the integer comparisons), infinite
    radii = [0.0, inst.d_cut / 3, inst.d_cut, 2.5 * inst.d_cut, 40000.0, math.inf]
    say(name, n, "radii", radii)
    rows = dpc.density_sweep(P, radii).cpu().numpy()
    for k, r in enumerate(radii):
        one = dpc.density(P, r).cpu().numpy()
        assert np.array_equal(rows[k], one), f"row {k} (d_cut {r})"
    assert np.all(rows[0] >= 1) and np.all(rows[-1] == n)
    assert np.all(np.diff(rows, axis=0) >= 0)  # density grows with the radius


def test_density_sweep_small_against_oracle():
    for seed, (n, d) in enumerate([(1, 2), (700, 1), (3000, 2), (2500, 5)]):
        p = datagen.clustered_small(40 + seed, n, d, span=1 << 14)
        radii = [0.0, 30.0, 300.0, 3000.0]
        rows = dpc.density_sweep(dev(p), radii).cpu().numpy()
        for k, r in enumerate(radii):
            want = oracle.run(p, r, 0, 0.0)[0]
            assert np.array_equal(rows[k], want), (n, d, r)


def test_cluster_sweep_rows_equal_single_calls_and_oracle():
    p = datagen.clustered_small(51, 6000, 2, span=1 << 16, k=6)
    d_cut = 900.0
    P = dev(p)
    rho, dep, d2, _ = dpc.run(P, d_cut, 0, 0.0)
    pairs = [(0, 0.0), (1, 1000.0), (5, 3600.0), (5, 10_000.0), (20, 3600.0), (50, 1e9), (0, math.inf)]
    rows = dpc.cluster_sweep(rho, dep, d2, pairs).cpu().numpy()
    for k, (rm, dm) in enumerate(pairs):
        one = dpc.cluster(rho, dep, d2, rm, dm).cpu().numpy()
        assert np.array_equal(rows[k], one), f"pair {k}"
        want = oracle.run(p, d_cut, rm, dm)[3]
        assert np.array_equal(rows[k], want), f"pair {k} against the oracle"


def test_cluster_sweep_checks_every_pair():
    p = datagen.clustered_small(52, 3000, 2, span=1 << 16)
    rho, dep, d2, _ = dpc.run(dev(p), 900.0, 0, 0.0)
    r, dp, dd = rho.cpu().numpy(), dep.cpu().numpy(), d2.cpu().numpy()
    # a non-root point with a finite delta: make its edge fall (point it at a
    # lower-priority point)
    order = np.lexsort((-np.arange(len(r)), r))  # ascending priority
    i = int(order[len(order) // 2])
    low = int(order[0])
    assert dp[i] >= 0 and low != i
    bad = dp.copy()
    bad[i] = low
    bad_t = torch.from_numpy(bad).cuda()
    # a pair that cuts the edge (delta_min at most delta) never follows it
    cut = (0, math.sqrt(float(dd[i])) * 0.5)
    follow = (0, math.inf)
    rows = dpc.cluster_sweep(rho, bad_t, d2, [cut]).cpu().numpy()
    assert np.array_equal(rows[0], dpc.cluster(rho, bad_t, d2, *cut).cpu().numpy())
    with pytest.raises(dpc.DPCError) as e:
        dpc.cluster_sweep(rho, bad_t, d2, [cut, follow])
    assert e.value.status == dpc._binding.ERR_NOT_FOREST
