"""Brute-force evaluation of the hoods' and the hull's definitions -- TEST
INFRASTRUCTURE.

For tiny inputs only.  Follows the paper's problem statement (the upper hood
of points in left-to-right order) and its orientation convention (r is left
of the directed segment pq iff det(q - p, r - p) > 0), with the readings used
throughout: vertical closure (only the highest point at an x can be a
corner, identical points resolve to the lowest index) and the strict hood
(points inside a hood edge are not corners).

Point i is a corner iff
  (i)  it is the representative of its x: no j with X_j = X_i and
       (Y_j > Y_i, or Y_j = Y_i and j < i); and
  (ii) no pair a, b with X_a < X_i < X_b has i on or below segment ab,
       i.e. det(b - a, i - a) <= 0.
Corners are returned in index order (which is left-to-right order).

Coordinates are converted to exact Python integers on the 2^-30 grid.
"""
from __future__ import annotations

import itertools

import numpy as np


def exact_ints(xy):
    a = np.asarray(xy, dtype=np.float32).reshape(-1, 2).astype(np.float64)
    s = a * float(1 << 30)
    if not np.all(np.floor(s) == s):
        raise ValueError("coordinate off the 2^-30 grid")
    X = [int(v) for v in s[:, 0]]
    Y = [int(v) for v in s[:, 1]]
    return X, Y


def det(X, Y, a, b, c) -> int:
    return (X[b] - X[a]) * (Y[c] - Y[a]) - (Y[b] - Y[a]) * (X[c] - X[a])


def upper_hull_brute(xy) -> list:
    X, Y = exact_ints(xy)
    n = len(X)
    out = []
    for i in range(n):
        rep = True
        for j in range(n):
            if j != i and X[j] == X[i] and (Y[j] > Y[i] or (Y[j] == Y[i] and j < i)):
                rep = False
                break
        if not rep:
            continue
        left = [a for a in range(n) if X[a] < X[i]]
        right = [b for b in range(n) if X[b] > X[i]]
        covered = False
        for a in left:
            for b in right:
                if det(X, Y, a, b, i) <= 0:
                    covered = True
                    break
            if covered:
                break
        if not covered:
            out.append(i)
    return out


def lower_hull_brute(xy) -> list:
    """The lower hood's definition, evaluated directly: point i is a corner
    iff it is the lowest point at its x (identical points: lowest index) and
    no pair a, b with X_a < X_i < X_b has i on or above segment ab."""
    X, Y = exact_ints(xy)
    n = len(X)
    out = []
    for i in range(n):
        if any(j != i and X[j] == X[i] and (Y[j] < Y[i] or (Y[j] == Y[i] and j < i))
               for j in range(n)):
            continue
        left = [a for a in range(n) if X[a] < X[i]]
        right = [b for b in range(n) if X[b] > X[i]]
        if not any(det(X, Y, a, b, i) >= 0 for a in left for b in right):
            out.append(i)
    return out


def _on_segment(X, Y, a, b, i) -> bool:
    return (det(X, Y, a, b, i) == 0 and min(X[a], X[b]) <= X[i] <= max(X[a], X[b])
            and min(Y[a], Y[b]) <= Y[i] <= max(Y[a], Y[b]))


def _in_triangle(X, Y, a, b, c, i) -> bool:
    d = det(X, Y, a, b, c)
    if d == 0:
        return False  # degenerate: covered by the segment test
    s = (det(X, Y, a, b, i), det(X, Y, b, c, i), det(X, Y, c, a, i))
    return all(v >= 0 for v in s) if d > 0 else all(v <= 0 for v in s)


def convex_hull_corners_brute(xy) -> list:
    """The corner set of the convex hull, from its definition: point i is a
    corner iff no identical point has a lower index and i does not lie in the
    closed convex hull of the points at other positions -- in the plane, iff
    it lies on no closed segment and in no closed triangle of such points
    (Caratheodory).  Returned in index order (the order around the hull is
    checked separately)."""
    X, Y = exact_ints(xy)
    n = len(X)
    out = []
    for i in range(n):
        if any(X[j] == X[i] and Y[j] == Y[i] for j in range(i)):
            continue
        others = [j for j in range(n) if X[j] != X[i] or Y[j] != Y[i]]
        inside = any(_on_segment(X, Y, a, b, i) for a, b in itertools.combinations(others, 2))
        if not inside:
            inside = any(_in_triangle(X, Y, a, b, c, i)
                         for a, b, c in itertools.combinations(others, 3))
        if not inside:
            out.append(i)
    return out
