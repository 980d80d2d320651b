"""Seeded synthetic inputs for exact Density Peaks Clustering.

This module only draws points: it holds none of the clustering arithmetic.
Both the CPU oracle (``oracle/``) and the GPU library are fed from here, so
the two sides see byte-identical int32 coordinates.

Every workload stands in for a data set of the paper's experiments (Section 7,
Table 2), which is not available here: the uniform / simden / varden sets of
10^7 2-D points, GeoLife-shaped 3-D data and HT-shaped 8-D data.  The recipes:

* ``blobs2d``   3 isotropic Gaussian blobs (sd 2,000) centred uniformly in
                [0, 1e5)^2 holding 95% of the points (multinomial, equal
                weights), plus 5% uniform noise in [0, 1e5)^2.  Rounded, not
                clipped.  d_cut 1,500, rho_min 20, delta_min 10,000.
* ``varden2d``  20 Gaussian clusters, sd log-uniform in [200, 20,000], weights
                Dirichlet(1), centres uniform in [0, 2^20)^2; 2% uniform noise;
                rounded and clipped to [0, 2^20).  d_cut calibrated for a
                median density of about 30; rho_min 5, delta_min 4 d_cut.
* ``uniform2d`` uniform integers in [0, 2^20)^2; mean density about 30.
* ``mix3d``     50% uniform in [0, 2^20)^3, 50% from 100 equal-weight clusters
                (sd 2^12); clipped; mean density about 50.
* ``aniso8d``   coordinates in [0, 2^16)^8: 50 anisotropic clusters (per-axis
                sd uniform in [2^8, 2^11]) plus 10% uniform noise; clipped;
                mean density about 50.

Every generator ends with a seeded shuffle of the point order, so input
indices carry no spatial information.  Random streams are numpy
``Generator(PCG64(SeedSequence(seed)))``.

The calibrated cut-off radii live in ``params.json`` next to this file; they
were written by ``oracle/calibrate_dcut.py`` (which only uses the oracle).  A
smaller instance of a recipe keeps the expected density by scaling the radius
with (n_full / n)^(1/d).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass

import numpy as np

__all__ = ["Instance", "WORKLOADS", "make", "random_small", "rng_for"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_PARAMS_PATH = os.path.join(_HERE, "params.json")


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


@dataclass
class Instance:
    name: str
    points: np.ndarray  # int32 [n, d], C-contiguous
    d_cut: float
    rho_min: int
    delta_min: float
    seed: int

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def d(self) -> int:
        return int(self.points.shape[1])


def _finish(rng, parts, lo, hi, clip):
    pts = np.concatenate(parts, axis=0)
    pts = np.rint(pts)
    if clip:
        np.clip(pts, lo, hi - 1, out=pts)
    pts = pts.astype(np.int64)
    perm = rng.permutation(pts.shape[0])
    return np.ascontiguousarray(pts[perm].astype(np.int32))


def _gaussian_clusters(rng, counts, centers, sds):
    parts = []
    for c, mu, sd in zip(counts, centers, sds):
        if c == 0:
            continue
        z = rng.standard_normal(size=(int(c), centers.shape[1]))
        z *= sd
        z += mu
        parts.append(z)
    return parts


def gen_blobs2d(n: int, seed: int) -> np.ndarray:
    rng = rng_for(seed)
    span = 100_000
    n_noise = int(round(0.05 * n))
    counts = rng.multinomial(n - n_noise, np.full(3, 1.0 / 3.0))
    centers = rng.uniform(0, span, size=(3, 2))
    parts = _gaussian_clusters(rng, counts, centers, np.full((3, 1), 2000.0))
    parts.append(rng.integers(0, span, size=(n_noise, 2)).astype(np.float64))
    return _finish(rng, parts, 0, span, clip=False)


def gen_varden2d(n: int, seed: int) -> np.ndarray:
    rng = rng_for(seed)
    span = 1 << 20
    k = 20
    sds = np.exp(rng.uniform(math.log(200.0), math.log(20_000.0), size=k))
    w = rng.dirichlet(np.ones(k))
    centers = rng.uniform(0, span, size=(k, 2))
    n_noise = int(round(0.02 * n))
    counts = rng.multinomial(n - n_noise, w)
    parts = _gaussian_clusters(rng, counts, centers, sds.reshape(k, 1))
    parts.append(rng.integers(0, span, size=(n_noise, 2)).astype(np.float64))
    return _finish(rng, parts, 0, span, clip=True)


def gen_uniform2d(n: int, seed: int) -> np.ndarray:
    rng = rng_for(seed)
    pts = rng.integers(0, 1 << 20, size=(n, 2)).astype(np.float64)
    return _finish(rng, [pts], 0, 1 << 20, clip=False)


def gen_mix3d(n: int, seed: int) -> np.ndarray:
    rng = rng_for(seed)
    span = 1 << 20
    k = 100
    n_uni = n // 2
    centers = rng.uniform(0, span, size=(k, 3))
    counts = rng.multinomial(n - n_uni, np.full(k, 1.0 / k))
    parts = _gaussian_clusters(rng, counts, centers, np.full((k, 1), float(1 << 12)))
    parts.append(rng.integers(0, span, size=(n_uni, 3)).astype(np.float64))
    return _finish(rng, parts, 0, span, clip=True)


def gen_aniso8d(n: int, seed: int) -> np.ndarray:
    rng = rng_for(seed)
    span = 1 << 16
    k = 50
    n_noise = int(round(0.10 * n))
    centers = rng.uniform(0, span, size=(k, 8))
    sds = rng.uniform(float(1 << 8), float(1 << 11), size=(k, 8))
    counts = rng.multinomial(n - n_noise, np.full(k, 1.0 / k))
    parts = _gaussian_clusters(rng, counts, centers, sds)
    parts.append(rng.integers(0, span, size=(n_noise, 8)).astype(np.float64))
    return _finish(rng, parts, 0, span, clip=True)


# name -> (generator, full n, d, seed, rho_min, delta_min factor or value,
#          fixed d_cut or None, calibration target)
WORKLOADS = {
    "blobs2d_10k": dict(gen=gen_blobs2d, n=10_000, d=2, seed=0, rho_min=20,
                        d_cut=1500.0, delta_min=10_000.0),
    "varden2d_1m": dict(gen=gen_varden2d, n=1_000_000, d=2, seed=1, rho_min=5,
                        target=("median", 30)),
    "varden2d_10m": dict(gen=gen_varden2d, n=10_000_000, d=2, seed=6, rho_min=5,
                         target=("median", 30)),
    "uniform2d_10m": dict(gen=gen_uniform2d, n=10_000_000, d=2, seed=7, rho_min=5,
                          target=("mean", 30)),
    "mix3d_10m": dict(gen=gen_mix3d, n=10_000_000, d=3, seed=2, rho_min=5,
                      target=("mean", 50)),
    "aniso8d_10m": dict(gen=gen_aniso8d, n=10_000_000, d=8, seed=3, rho_min=5,
                        target=("mean", 50)),
}


def _load_params() -> dict:
    if not os.path.exists(_PARAMS_PATH):
        return {}
    with open(_PARAMS_PATH) as f:
        return json.load(f)


def full_d_cut(name: str) -> float | None:
    spec = WORKLOADS[name]
    if "d_cut" in spec:
        return float(spec["d_cut"])
    return _load_params().get(name, {}).get("d_cut")


def make(name: str, n: int | None = None, seed: int | None = None,
         d_cut: float | None = None) -> Instance:
    """Draw workload ``name`` with ``n`` points (default: its full size).

    The radius defaults to the calibrated full-size radius, scaled by
    (n_full / n)^(1/d) for a smaller draw of the same recipe so that the
    expected density stays about the same.
    """
    spec = WORKLOADS[name]
    n_full = spec["n"]
    n = n_full if n is None else int(n)
    seed = spec["seed"] if seed is None else int(seed)
    pts = spec["gen"](n, seed)
    if d_cut is None:
        base = full_d_cut(name)
        if base is None:
            raise RuntimeError(f"no calibrated d_cut for {name}; run oracle/calibrate_dcut.py")
        d_cut = float(base) * (n_full / n) ** (1.0 / spec["d"]) if n != n_full else float(base)
        if n != n_full and "d_cut" not in spec:
            d_cut = float(math.floor(d_cut))
    if "delta_min" in spec:
        delta_min = float(spec["delta_min"])
    else:
        delta_min = 4.0 * d_cut
    return Instance(name=name, points=pts, d_cut=float(d_cut), rho_min=int(spec["rho_min"]),
                    delta_min=delta_min, seed=seed)


def random_small(seed: int, n: int, d: int, span: int, offset: int = 0) -> np.ndarray:
    """Uniform integer points in [offset, offset + span)^d.

    A small span forces duplicate points and ties in both density and
    distance, which is what the tie-breaking tests need.
    """
    rng = rng_for(seed)
    pts = rng.integers(offset, offset + span, size=(n, d), dtype=np.int64)
    return np.ascontiguousarray(pts.astype(np.int32))


def clustered_small(seed: int, n: int, d: int, span: int = 1 << 20, k: int = 5,
                    sd_frac: float = 0.02, noise: float = 0.05) -> np.ndarray:
    """A few Gaussian blobs plus uniform noise, rounded and clipped to [0, span)."""
    rng = rng_for(seed)
    n_noise = int(round(noise * n))
    centers = rng.uniform(0, span, size=(k, d))
    counts = rng.multinomial(n - n_noise, np.full(k, 1.0 / k))
    parts = _gaussian_clusters(rng, counts, centers, np.full((k, 1), sd_frac * span))
    parts.append(rng.integers(0, span, size=(n_noise, d)).astype(np.float64))
    return _finish(rng, parts, 0, span, clip=True)


# ---------------------------------------------------------------------------
# many independent instances (batched and served workloads)

def _dcut_for_median_rho(points: np.ndarray, target: int, rng, sample: int = 256) -> float:
    """A radius giving a median density of about ``target`` (self included):
    the median distance from a sample of points to their ``target``-th
    nearest neighbour (counting the point itself), from scipy's k-d tree.
    This only sets an input parameter; no output is derived from it."""
    from scipy.spatial import cKDTree

    n = points.shape[0]
    k = min(target, n)
    idx = rng.choice(n, size=min(sample, n), replace=False)
    dist, _ = cKDTree(points.astype(np.float64)).query(points[idx].astype(np.float64), k=k)
    dk = dist[:, -1] if dist.ndim == 2 else dist
    return float(max(np.median(dk), 1.0))


def gen_blob_instance(rng, n: int, d: int, span: int = 1 << 20, noise: float = 0.05) -> np.ndarray:
    """2-50 isotropic Gaussian blobs (sd span/50, equal weights) plus uniform
    noise, rounded and clipped to [0, span)^d."""
    k = int(rng.integers(2, 51))
    n_noise = int(round(noise * n))
    centers = rng.uniform(0, span, size=(k, d))
    counts = rng.multinomial(n - n_noise, np.full(k, 1.0 / k))
    parts = _gaussian_clusters(rng, counts, centers, np.full((k, 1), span / 50.0))
    parts.append(rng.integers(0, span, size=(n_noise, d)).astype(np.float64))
    return _finish(rng, parts, 0, span, clip=True)


def gen_uniform_instance(rng, n: int, d: int, span: int = 1 << 20) -> np.ndarray:
    pts = rng.integers(0, span, size=(n, d), dtype=np.int64)
    return np.ascontiguousarray(pts.astype(np.int32))


def batch_instances(seed: int = 4, count: int = 512, n_lo: int = 1_000, n_hi: int = 200_000,
                    dims=(2, 3, 5, 8), median_rho: int = 20) -> list:
    """The batched workload: ``count`` independent instances, n log-uniform in
    [n_lo, n_hi], d uniform over ``dims``, Gaussian-blob data (2-50 blobs, 5%
    noise, [0, 2^20)^d), d_cut for a median density of about 20, rho_min 5,
    delta_min 4 d_cut.  Instance i draws from seed (seed, i)."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, i])))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(dims[int(rng.integers(0, len(dims)))])
        pts = gen_blob_instance(rng, n, d)
        d_cut = _dcut_for_median_rho(pts, median_rho, rng)
        out.append(Instance(name=f"batch{seed}_{i}", points=pts, d_cut=d_cut, rho_min=5,
                            delta_min=4.0 * d_cut, seed=seed))
    return out


def served_instances(seed: int = 5, count: int = 64, n_lo: int = 1_000, n_hi: int = 1_000_000, d: int = 3,
                     median_rho: int = 20) -> list:
    """The request pool of the served workload: n log-uniform in [n_lo, n_hi],
    d = 3, each uniform or Gaussian blobs with probability 1/2, int32 in
    [0, 2^20)^3; parameters as in the batched workload.  A request stream
    draws its requests from this pool."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, i])))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        if rng.random() < 0.5:
            pts = gen_uniform_instance(rng, n, d)
        else:
            pts = gen_blob_instance(rng, n, d)
        d_cut = _dcut_for_median_rho(pts, median_rho, rng)
        out.append(Instance(name=f"served{seed}_{i}", points=pts, d_cut=d_cut, rho_min=5,
                            delta_min=4.0 * d_cut, seed=seed))
    return out
