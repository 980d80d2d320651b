"""Pure-Python DPC for tiny inputs: a second, independent oracle.

TEST INFRASTRUCTURE ONLY (see the C oracle's header).  It uses Python's
unbounded integers and exact rationals, and loops over every pair, so it is
meant for a few hundred points at most.  The C oracle is checked against it.

Definitions 1-5 of Section 3 and Algorithm 3 of Section 6.2, with the same
readings as the C oracle: closed ball, priority (rho, -index), distance ties
to the smaller index, dep = -1 / delta^2 = INT64_MAX for the top point,
label = index of the centre reached, -1 for noise.
"""
from __future__ import annotations

import math
from fractions import Fraction

INF = (1 << 63) - 1


def square_threshold(r: float, round_up: bool) -> int:
    """floor(r^2) or ceil(r^2) of the exact rational value of the double r."""
    if math.isnan(r) or r < 0:
        raise ValueError("radius must be a non-negative number")
    if math.isinf(r):
        return INF
    sq = Fraction(r) ** 2
    v = math.ceil(sq) if round_up else math.floor(sq)
    return min(v, INF)


def delta_threshold(delta_min: float) -> int:
    if math.isnan(delta_min):
        raise ValueError("delta_min is NaN")
    if delta_min <= 0:
        return 0
    return square_threshold(delta_min, True)


def sqd(p, q) -> int:
    return sum((int(a) - int(b)) ** 2 for a, b in zip(p, q))


def density(points, T: int):
    pts = [tuple(int(v) for v in p) for p in points]
    return [sum(1 for q in pts if sqd(p, q) <= T) for p in pts]


def above(rho, j, i) -> bool:
    return (rho[j], -j) > (rho[i], -i)


def dependent(points, rho, rho_min: int = 0, skip_noise: bool = False):
    pts = [tuple(int(v) for v in p) for p in points]
    n = len(pts)
    dep, d2 = [], []
    for i in range(n):
        if skip_noise and rho[i] < rho_min:
            dep.append(-1)
            d2.append(INF)
            continue
        cands = [(sqd(pts[i], pts[j]), j) for j in range(n) if above(rho, j, i)]
        if cands:
            dist, j = min(cands)
            dep.append(j)
            d2.append(dist)
        else:
            dep.append(-1)
            d2.append(INF)
    return dep, d2


def cluster(rho, dep, delta2, rho_min: int, Td: int):
    labels = []
    for i in range(len(rho)):
        if rho[i] < rho_min:
            labels.append(-1)
            continue
        c = i
        while delta2[c] < Td:
            p = dep[c]
            if p < 0 or not above(rho, p, c):
                raise ValueError("not a dependent forest")
            c = p
        labels.append(c)
    return labels


def run(points, d_cut: float, rho_min: int, delta_min: float, skip_noise: bool = False):
    T = square_threshold(d_cut, False)
    Td = delta_threshold(delta_min)
    rho = density(points, T)
    dep, d2 = dependent(points, rho, rho_min, skip_noise)
    lab = cluster(rho, dep, d2, rho_min, Td)
    return rho, dep, d2, lab
