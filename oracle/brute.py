"""O(n^3) evaluation of the upper hood's definition -- TEST INFRASTRUCTURE.

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
