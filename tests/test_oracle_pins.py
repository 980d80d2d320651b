"""Pins for the CPU oracle: it is checked against things other than itself.

* hand-worked examples (tests/golden, derived from Section 3's definitions);
* exact rational arithmetic for the threshold conversion;
* an independent pure-Python oracle on thousands of tiny random inputs;
* scipy's k-d tree ball counts (a library routine the oracle does not use);
* closed forms: d_cut = 0 (multiplicity), d_cut >= diameter (prefix nearest
  neighbour), unit lattices (3/4/5 and 4/6/9 neighbour counts);
* a textbook reduction: on a line, the dependent point is the nearer of the
  all-nearest-larger-values to the left and right (monotone stack);
* invariants of the dependent forest and the labels;
* metamorphic relations (translation, axis permutation, reflection, scaling);
* planted mistakes in a copy of the Python oracle are caught by the pins.
"""
import glob
import json
import math
import os
import random
import struct

import numpy as np
import pytest
from fractions import Fraction

import datagen
import oracle
from oracle import ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INF = oracle.INF


def _load_golden(path):
    with open(path) as f:
        g = json.load(f)
    g["delta2"] = [INF if v == "INF" else int(v) for v in g["delta2"]]
    return g


GOLDEN_FILES = sorted(glob.glob(os.path.join(GOLDEN, "*.json")))


@pytest.mark.parametrize("path", GOLDEN_FILES, ids=[os.path.basename(p) for p in GOLDEN_FILES])
def test_golden_c_oracle(path):
    g = _load_golden(path)
    pts = np.array(g["points"], np.int32)
    rho, dep, d2, lab = oracle.run(pts, g["d_cut"], g["rho_min"], g["delta_min"], g["skip_noise"])
    assert rho.tolist() == g["rho"]
    assert dep.tolist() == g["dep"]
    assert d2.tolist() == g["delta2"]
    assert lab.tolist() == g["label"]


@pytest.mark.parametrize("path", GOLDEN_FILES, ids=[os.path.basename(p) for p in GOLDEN_FILES])
def test_golden_python_oracle(path):
    g = _load_golden(path)
    rho, dep, d2, lab = ref.run(g["points"], g["d_cut"], g["rho_min"], g["delta_min"], g["skip_noise"])
    assert rho == g["rho"] and dep == g["dep"] and d2 == g["delta2"] and lab == g["label"]


def test_golden_skip_mode_labels_unchanged():
    # The labels do not depend on whether noise points get a dependent.
    for path in GOLDEN_FILES:
        g = _load_golden(path)
        pts = np.array(g["points"], np.int32)
        a = oracle.run(pts, g["d_cut"], g["rho_min"], g["delta_min"], False)
        b = oracle.run(pts, g["d_cut"], g["rho_min"], g["delta_min"], True)
        assert a[3].tolist() == b[3].tolist()
        assert a[0].tolist() == b[0].tolist()


# ----------------------------------------------------------------------------
# thresholds: floor(d_cut^2) and ceil(delta_min^2) of the exact double value


def _exact(r, up):
    if math.isinf(r):
        return INF
    v = Fraction(r) ** 2
    v = math.ceil(v) if up else math.floor(v)
    return min(v, INF)


THRESHOLD_CASES = [
    0.0, 5e-324, 0.25, 0.5, 0.9999999999999999, 1.0, 1.0000000000000002, 1.5,
    math.sqrt(2.0), math.sqrt(3.0), 30.0, 1500.0, 1500.0000000000002, 1499.9999999999998,
    2.0 ** 26, 2.0 ** 26.5, 94906265.62425154, 2.0 ** 31.5, 3037000499.97605,
    3037000499.0, 3037000500.0, 2.0 ** 40, 1e300, math.inf,
]


@pytest.mark.parametrize("r", THRESHOLD_CASES)
def test_square_threshold_exact(r):
    assert oracle.square_threshold(r, False) == _exact(r, False)
    if r != math.inf:
        assert oracle.square_threshold(r, True) == _exact(r, True)
    assert ref.square_threshold(r, False) == _exact(r, False)


def test_square_threshold_known_values():
    assert oracle.square_threshold(1500.0) == 2_250_000
    assert oracle.square_threshold(math.sqrt(2.0)) == 2  # 2.0000000000000004 rounds down
    assert oracle.square_threshold(math.sqrt(2.0), True) == 3
    assert oracle.square_threshold(0.5) == 0 and oracle.square_threshold(0.5, True) == 1
    assert oracle.square_threshold(3037000499.0) == 3037000499 ** 2
    assert oracle.square_threshold(3037000500.0) == INF  # 3037000500^2 > 2^63 - 1
    assert oracle.delta_threshold(-1.0) == 0 and oracle.delta_threshold(0.0) == 0
    with pytest.raises(ValueError):
        oracle.square_threshold(-1.0)
    with pytest.raises(ValueError):
        oracle.square_threshold(float("nan"))


def test_square_threshold_random_doubles():
    rng = random.Random(1234)
    for _ in range(4000):
        bits = rng.getrandbits(64) & 0x7FEFFFFFFFFFFFFF  # finite, non-negative
        r = struct.unpack("<d", struct.pack("<Q", bits))[0]
        if rng.random() < 0.5:
            r = rng.uniform(0, 2.0 ** rng.randint(-4, 33))
        assert oracle.square_threshold(r, False) == _exact(r, False)
        assert oracle.square_threshold(r, True) == _exact(r, True)


# ----------------------------------------------------------------------------
# the C oracle against the pure-Python oracle on tiny inputs full of ties


def test_c_oracle_matches_python_oracle_random():
    rng = random.Random(99)
    for case in range(600):
        n = rng.randint(1, 36)
        d = rng.randint(1, 4)
        span = rng.choice([2, 3, 5, 8, 20, 1000])
        pts = datagen.random_small(case, n, d, span, offset=rng.randint(-50, 50))
        d_cut = rng.choice([0.0, 1.0, math.sqrt(2.0), 2.5, 4.0, float(span), rng.uniform(0, span)])
        rho_min = rng.randint(0, 4)
        delta_min = rng.choice([0.0, 1.0, 1.5, 3.0, rng.uniform(0, 2 * span), math.inf])
        skip = rng.random() < 0.5
        a = oracle.run(pts, d_cut, rho_min, delta_min, skip)
        b = ref.run(pts.tolist(), d_cut, rho_min, delta_min, skip)
        for x, y in zip(a, b):
            assert x.tolist() == list(y), (case, n, d, span, d_cut)


def test_per_query_forms_match_python_oracle():
    """density_at and dependent_at (the references of the full-size GPU
    checks) against the pure-Python oracle on tie-heavy inputs, with query
    lists in random order and with repeats, radii 0 and infinity included
    (Section 3, Definitions 1-3)."""
    rng = random.Random(7)
    for case in range(300):
        n = rng.randint(1, 40)
        d = rng.randint(1, 5)
        span = rng.choice([2, 3, 5, 8, 20])
        pts = datagen.random_small(1000 + case, n, d, span, offset=rng.randint(-20, 20))
        d_cut = rng.choice([0.0, math.inf, 1.0, math.sqrt(2.0), rng.uniform(0, span)])
        T = ref.square_threshold(d_cut, False)
        want_rho = ref.density(pts.tolist(), T)
        q = [rng.randrange(n) for _ in range(rng.randint(1, 2 * n))]
        assert oracle.density_at(pts, T, np.array(q, np.int64)).tolist() == [want_rho[i] for i in q], case
        # arbitrary densities (few distinct values) exercise the priority ties
        rho = [rng.randint(1, 3) for _ in range(n)]
        wd, wd2 = ref.dependent(pts.tolist(), rho)
        gd, gd2 = oracle.dependent_at(pts, np.array(rho, np.int32), np.array(q, np.int64))
        assert gd.tolist() == [wd[i] for i in q] and gd2.tolist() == [wd2[i] for i in q], case


# ----------------------------------------------------------------------------
# density against scipy's k-d tree (an independent library routine)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
def test_density_matches_scipy_kdtree(d):
    from scipy.spatial import cKDTree

    pts = datagen.clustered_small(7 + d, 1500, d, span=4000, k=4, sd_frac=0.05)
    T = oracle.square_threshold(150.0 * math.sqrt(d))
    rho = oracle.density(pts, T)
    # D^2 is an integer, so D^2 <= T  <=>  D <= sqrt(T + 1/2): no boundary rounding issue.
    tree = cKDTree(pts.astype(np.float64))
    cnt = tree.query_ball_point(pts.astype(np.float64), r=math.sqrt(T + 0.5), return_length=True)
    assert rho.tolist() == list(np.asarray(cnt, dtype=np.int64))


def test_density_pair_count_identity():
    from scipy.spatial.distance import pdist

    pts = datagen.clustered_small(3, 1200, 3, span=2000, k=3, sd_frac=0.05)
    T = 80 ** 2
    rho = oracle.density(pts, T)
    pairs = int(np.count_nonzero(pdist(pts.astype(np.float64), "sqeuclidean") <= T))
    assert int(rho.sum()) == pts.shape[0] + 2 * pairs
    assert rho.min() >= 1


# ----------------------------------------------------------------------------
# closed forms


def test_dcut_zero_is_multiplicity():
    pts = datagen.random_small(5, 400, 2, 6)
    rho = oracle.density(pts, 0)
    _, inv, counts = np.unique(pts, axis=0, return_inverse=True, return_counts=True)
    assert rho.tolist() == counts[inv.reshape(-1)].tolist()


def test_dcut_beyond_diameter_is_prefix_nearest_neighbour():
    pts = datagen.random_small(6, 300, 3, 50)
    n = pts.shape[0]
    rho, dep, d2, _ = oracle.run(pts, 1e6, 0, 0.0)
    assert (rho == n).all()
    # Every density is n, so j ranks above i exactly when j < i: the dependent
    # point is the nearest earlier point, ties to the smaller index.
    P = pts.astype(np.int64)
    assert dep[0] == -1 and d2[0] == INF
    for i in range(1, n):
        dd = ((P[:i] - P[i]) ** 2).sum(axis=1)
        j = int(np.lexsort((np.arange(i), dd))[0])
        assert dep[i] == j and d2[i] == dd[j]


@pytest.mark.parametrize("k", [3, 4, 5, 7])
def test_unit_lattice_counts(k):
    pts = np.array([[x, y] for y in range(k) for x in range(k)], np.int32)
    rho1 = oracle.density(pts, 1).reshape(k, k)
    rho2 = oracle.density(pts, 2).reshape(k, k)
    for y in range(k):
        for x in range(k):
            border = (x in (0, k - 1)) + (y in (0, k - 1))
            assert rho1[y, x] == {0: 5, 1: 4, 2: 3}[border]
            assert rho2[y, x] == {0: 9, 1: 6, 2: 4}[border]


# ----------------------------------------------------------------------------
# reduction to all-nearest-larger-values on a line


def _ansv_dependents(xs, rho):
    """Nearest higher-priority point on a line by two monotone-stack passes."""
    n = len(xs)
    order = sorted(range(n), key=lambda i: xs[i])
    key = [(rho[i], -i) for i in range(n)]
    left = [None] * n
    right = [None] * n
    stack = []
    for i in order:
        while stack and key[stack[-1]] < key[i]:
            stack.pop()
        left[i] = stack[-1] if stack else None
        stack.append(i)
    stack = []
    for i in reversed(order):
        while stack and key[stack[-1]] < key[i]:
            stack.pop()
        right[i] = stack[-1] if stack else None
        stack.append(i)
    out = []
    for i in range(n):
        c = [(abs(xs[i] - xs[j]) ** 2, j) for j in (left[i], right[i]) if j is not None]
        out.append(min(c) if c else (INF, -1))
    return out


@pytest.mark.parametrize("d", [1, 2])
def test_line_reduces_to_ansv(d):
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(2, 300))
        xs = rng.choice(np.arange(-5000, 5000), size=n, replace=False)
        pts = np.zeros((n, d), np.int32)
        pts[:, 0] = xs
        d_cut = float(rng.choice([0.0, 10.0, 40.0, 200.0]))
        rho = oracle.density(pts, oracle.square_threshold(d_cut))
        dep, d2 = oracle.dependent(pts, rho)
        expect = _ansv_dependents([int(x) for x in xs], rho.tolist())
        assert [(int(a), int(b)) for a, b in zip(d2, dep)] == expect


# ----------------------------------------------------------------------------
# invariants of the forest and the labels


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forest_and_label_invariants(seed):
    pts = datagen.clustered_small(seed, 2500, 2, span=20000, k=4, sd_frac=0.03, noise=0.1)
    d_cut, rho_min, delta_min = 300.0, 4, 1500.0
    rho, dep, d2, lab = oracle.run(pts, d_cut, rho_min, delta_min)
    n = pts.shape[0]
    P = pts.astype(np.int64)
    Td = oracle.delta_threshold(delta_min)
    key = rho.astype(np.int64) * (1 << 32) + ((1 << 32) - 1 - np.arange(n))
    roots = np.flatnonzero(dep < 0)
    assert roots.tolist() == [int(np.argmax(key))]  # the lowest-index maximum-density point
    assert d2[roots[0]] == INF
    nz = dep >= 0
    assert (key[dep[nz]] > key[nz]).all()
    assert (d2[nz] == ((P[nz] - P[dep[nz]]) ** 2).sum(axis=1)).all()
    noise = rho < rho_min
    assert ((lab == -1) == noise).all()
    centre = (~noise) & (d2 >= Td)
    assert (lab[centre] == np.flatnonzero(centre)).all()
    follow = (~noise) & (d2 < Td)
    assert (lab[follow] == lab[dep[follow]]).all()
    assert len(set(lab[~noise].tolist())) == int(centre.sum())


def test_raising_thresholds_coarsens_and_keeps_labels():
    pts = datagen.clustered_small(4, 2000, 2, span=20000, k=5, sd_frac=0.03)
    rho, dep, d2, lab1 = oracle.run(pts, 300.0, 3, 1000.0)
    _, _, _, lab2 = oracle.run(pts, 300.0, 3, 4000.0)
    # a larger delta_min merges clusters: equal labels stay equal
    for a in np.unique(lab1[lab1 >= 0]):
        assert len(np.unique(lab2[lab1 == a])) == 1
    _, _, _, lab3 = oracle.run(pts, 300.0, 6, 1000.0)
    keep = rho >= 6
    assert (lab3[keep] == lab1[keep]).all() and (lab3[~keep] == -1).all()


# ----------------------------------------------------------------------------
# metamorphic relations


def test_metamorphic_relations():
    pts = datagen.clustered_small(8, 1200, 3, span=5000, k=3, sd_frac=0.05)
    base = oracle.run(pts, 200.0, 3, 700.0)
    moved = oracle.run(pts + np.array([123, -77, 5000], np.int32), 200.0, 3, 700.0)
    perm = oracle.run(np.ascontiguousarray(pts[:, [2, 0, 1]]), 200.0, 3, 700.0)
    refl = oracle.run(np.ascontiguousarray(pts * np.array([1, -1, 1], np.int32)), 200.0, 3, 700.0)
    for other in (moved, perm, refl):
        for x, y in zip(base, other):
            assert (x == y).all()
    scaled = oracle.run(pts * 3, 600.0, 3, 2100.0)
    assert (scaled[0] == base[0]).all() and (scaled[1] == base[1]).all()
    nz = base[1] >= 0
    assert (scaled[2][nz] == 9 * base[2][nz]).all()
    assert (scaled[3] == base[3]).all()


def test_reordering_is_not_an_invariance_with_ties():
    # Ties are broken by index, so reversing the order of identical points
    # changes which copy is the root: a negative check on the tie rule.
    pts = np.zeros((4, 2), np.int32)
    a = oracle.run(pts, 0.0, 1, 1.0)
    assert a[1].tolist() == [-1, 0, 0, 0]


# ----------------------------------------------------------------------------
# range check and forest validation


def test_range_check_boundary():
    w = 3037000499  # w^2 <= 2^63 - 1 < (w + 1)^2
    lo = -1518500249
    ok = np.array([[lo], [lo + w]], np.int32)
    bad = np.array([[lo], [lo + w + 1]], np.int32)
    assert oracle.range_ok(ok) and not oracle.range_ok(bad)
    two = np.array([[-(2 ** 31), -(2 ** 31)], [2 ** 31 - 1, 2 ** 31 - 1]], np.int32)
    assert not oracle.range_ok(two)
    with pytest.raises(ValueError):
        oracle.run(bad, 1.0, 0, 1.0)
    rho, dep, d2, _ = oracle.run(ok, 1.0, 0, 1.0)
    assert d2.tolist() == [INF, w * w]


def test_cluster_rejects_non_forest():
    rho = np.array([2, 2, 2], np.int32)
    d2 = np.array([1, 1, 1], np.int64)
    with pytest.raises(ValueError):
        oracle.cluster(rho, np.array([1, 2, 0], np.int32), d2, 0, 5)  # cycle
    with pytest.raises(ValueError):
        oracle.cluster(rho, np.array([-1, 2, 0], np.int32), d2, 0, 5)  # 1 -> 2 ranks lower
    lab = oracle.cluster(rho, np.array([-1, 0, 0], np.int32), np.array([INF, 1, 1], np.int64), 0, 5)
    assert lab.tolist() == [0, 0, 0]


# ----------------------------------------------------------------------------
# planted mistakes in a copy of the Python oracle must fail a pin


def _mutant_run(points, d_cut, rho_min, delta_min, skip, mutation):
    T = ref.square_threshold(d_cut, False)
    Td = ref.delta_threshold(delta_min)
    pts = [tuple(int(v) for v in p) for p in points]
    n = len(pts)
    if mutation == "open_ball":
        rho = [sum(1 for q in pts if ref.sqd(p, q) < T) for p in pts]
    elif mutation == "no_self":
        rho = [sum(1 for j, q in enumerate(pts) if j != i and ref.sqd(p, q) <= T) for i, p in enumerate(pts)]
    elif mutation == "dropped_axis":
        rho = [sum(1 for q in pts if (p[0] - q[0]) ** 2 <= T) for p in pts]
    else:
        rho = ref.density(points, T)

    def above(j, i):
        if mutation == "density_tie_high_index":
            return (rho[j], j) > (rho[i], i)
        return (rho[j], -j) > (rho[i], -i)

    dep, d2 = [], []
    for i in range(n):
        if skip and rho[i] < rho_min:
            dep.append(-1)
            d2.append(INF)
            continue
        c = [(ref.sqd(pts[i], pts[j]), -j if mutation == "distance_tie_high_index" else j)
             for j in range(n) if above(j, i)]
        if c:
            dist, j = min(c)
            j = abs(j)
            dep.append(j)
            d2.append(dist)
        else:
            dep.append(-1)
            d2.append(INF)
    lab = []
    for i in range(n):
        if rho[i] < rho_min:
            lab.append(-1)
            continue
        c = i
        while (d2[c] <= Td) if mutation == "centre_strict" else (d2[c] < Td):
            if dep[c] < 0:
                break
            c = dep[c]
        lab.append(c)
    return rho, dep, d2, lab


@pytest.mark.parametrize("mutation", ["open_ball", "no_self", "dropped_axis", "density_tie_high_index",
                                      "distance_tie_high_index", "centre_strict"])
def test_pins_catch_planted_mistakes(mutation):
    caught = False
    for path in GOLDEN_FILES:
        g = _load_golden(path)
        got = _mutant_run(g["points"], g["d_cut"], g["rho_min"], g["delta_min"], g["skip_noise"], mutation)
        if list(got) != [g["rho"], g["dep"], g["delta2"], g["label"]]:
            caught = True
    assert caught, mutation
