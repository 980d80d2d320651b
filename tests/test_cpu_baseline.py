"""The multithreaded CPU baseline (cpu_baseline/) against the oracle.

bench.py times it beside the GPU library and compares their outputs at full
size, so it must be exact: every output equals the oracle's on small inputs
full of ties, at several thread counts.
"""
import math

import numpy as np
import pytest

import cpu_baseline
import datagen
import oracle


@pytest.fixture(scope="module", autouse=True)
def _built():
    cpu_baseline.build()


def same(a, b, what):
    for name, x, y in zip(("rho", "dep", "delta2", "label"), a, b):
        assert np.array_equal(x, y), f"{what}: {name}"


def test_random_tiny_against_oracle():
    rng = np.random.default_rng(70)
    for t in range(300):
        d = int(rng.integers(1, 9))
        n = int(rng.integers(1, 300))
        span = int(rng.choice([2, 5, 40, 3000]))
        p = datagen.random_small(int(rng.integers(1 << 30)), n, d, span)
        dc = float(rng.choice([0.0, 1.0, 1.5, 7.0, 60.0, math.inf]))
        rm = int(rng.integers(0, 6))
        dm = float(rng.choice([0.0, 1.0, 2.5, 30.0, math.inf]))
        same(cpu_baseline.run(p, dc, rm, dm, threads=int(rng.integers(1, 6))), oracle.run(p, dc, rm, dm),
             f"case {t} n={n} d={d} span={span}")


@pytest.mark.parametrize("name,n", [("blobs2d_10k", 10_000), ("varden2d_1m", 8000), ("mix3d_10m", 8000),
                                    ("aniso8d_10m", 4000)])
def test_workload_shapes_against_oracle(name, n):
    x = datagen.make(name, n=n)
    same(cpu_baseline.run(x.points, x.d_cut, x.rho_min, x.delta_min, threads=4),
         oracle.run(x.points, x.d_cut, x.rho_min, x.delta_min), name)


def test_wide_coordinates_and_range_error():
    p = datagen.random_small(3, 500, 2, 1 << 20)
    p[:2] = [[-2**29, -2**29], [2**29, 2**29]]  # squared spans beyond 2^53: int64 distances
    same(cpu_baseline.run(p, 1e6, 2, 3e6), oracle.run(p, 1e6, 2, 3e6), "wide")
    wide = np.array([[0, 0], [2**31 - 1, 2**31 - 1], [-2**31, -2**31]], np.int32)
    with pytest.raises(RuntimeError):
        cpu_baseline.run(wide, 1.0, 0, 1.0)
