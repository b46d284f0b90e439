"""Exact invariants of the strict upper hood (and of the lower hood and the
convex hull) -- TEST INFRASTRUCTURE.

``check(xy, idx)`` returns a list of violated properties (empty when the
index list is exactly the strict upper hood of xy).  Together the checks
characterise the answer uniquely: a strictly concave chain through input
points, from the representative of the smallest x to that of the largest x,
with every input point on or below it, is the upper hood's boundary, and the
strict-turn condition fixes its corner set.

All arithmetic is exact int64 on the 2^-30 grid: with x in [0, 1] and y in
[-1, 1], every product is below 2^61 and every determinant below 2^62.
"""
from __future__ import annotations

import numpy as np


def _grid(xy):
    a = np.asarray(xy, dtype=np.float32).reshape(-1, 2).astype(np.float64)
    s = a * float(1 << 30)
    if not np.all(np.floor(s) == s):
        raise ValueError("coordinate off the 2^-30 grid")
    if a.size and (a[:, 0].min() < 0 or a[:, 0].max() > 1
                   or a[:, 1].min() < -1 or a[:, 1].max() > 1):
        raise ValueError("coordinate out of range")
    return s[:, 0].astype(np.int64), s[:, 1].astype(np.int64)


def _det(ax, ay, bx, by, cx, cy):
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)


def check(xy, idx) -> list:
    X, Y = _grid(xy)
    n = X.shape[0]
    h = np.asarray(idx, dtype=np.int64)
    errs = []
    if n == 0:
        return [] if h.size == 0 else ["non-empty output for empty input"]
    if h.size == 0:
        return ["empty output for non-empty input"]
    if h.min() < 0 or h.max() >= n:
        return ["index out of range"]
    if np.any(np.diff(h) <= 0):
        errs.append("indices not strictly increasing")
    HX, HY = X[h], Y[h]
    if np.any(np.diff(HX) <= 0):
        errs.append("corner x not strictly increasing")
    # representative of an x: max y, then lowest index
    order = np.lexsort((np.arange(n), -Y, X))  # by x, then y desc, then index
    first_of_x = np.ones(n, dtype=bool)
    first_of_x[1:] = X[order][1:] != X[order][:-1]
    reps = np.sort(order[first_of_x])
    is_rep = np.zeros(n, dtype=bool)
    is_rep[reps] = True
    if not np.all(is_rep[h]):
        errs.append("a corner is not the representative of its x")
    if h[0] != reps[0]:
        errs.append("first corner is not the representative of the smallest x")
    if h[-1] != reps[-1]:
        errs.append("last corner is not the representative of the largest x")
    if h.size >= 3:
        d = _det(HX[:-2], HY[:-2], HX[1:-1], HY[1:-1], HX[2:], HY[2:])
        if np.any(d >= 0):
            errs.append("chain not strictly concave (a corner is not a strict turn)")
    if errs:
        return errs
    # every point on or below the edge spanning its x
    k = np.searchsorted(HX, X, side="right") - 1  # HX[k] <= X < HX[k+1]
    k = np.clip(k, 0, max(h.size - 2, 0))
    if h.size >= 2:
        a, b = h[k], h[k + 1]
        d = _det(X[a], Y[a], X[b], Y[b], X, Y)
        if np.any(d > 0):
            errs.append("an input point lies strictly above the chain")
    else:
        if np.any(X != HX[0]):
            errs.append("single corner but points at other x")
        if np.any(Y > HY[0]):
            errs.append("a point lies above the single corner")
    return errs


def check_lower(xy, idx) -> list:
    """``check`` for the lower hood: the lower hood of a set is the upper
    hood of its mirror image under y -> -y, with the same indices."""
    a = np.asarray(xy, dtype=np.float32).reshape(-1, 2).copy()
    a[:, 1] = -a[:, 1]
    return check(a, idx)


def check_convex_hull(xy, idx) -> list:
    """Violated properties of a counter-clockwise convex-hull corner list.

    A polygon through input points that turns strictly left at every corner
    and has every input point on or left of every edge is the convex hull
    with exactly its corners; starting at the lowest point of least x (lowest
    index among identical points) fixes the order."""
    X, Y = _grid(xy)
    n = X.shape[0]
    h = np.asarray(idx, dtype=np.int64)
    if n == 0:
        return [] if h.size == 0 else ["non-empty output for empty input"]
    if h.size == 0:
        return ["empty output for non-empty input"]
    if h.min() < 0 or h.max() >= n:
        return ["index out of range"]
    errs = []
    if np.unique(h).size != h.size:
        errs.append("an index appears twice")
    start = np.lexsort((np.arange(n), Y, X))[0]  # least x, then least y, then index
    if h[0] != start:
        errs.append("does not start at the lowest point of least x")
    first_copy = {}
    for i in range(n):
        first_copy.setdefault((int(X[i]), int(Y[i])), i)
    if any(first_copy[(int(X[i]), int(Y[i]))] != i for i in h):
        errs.append("a corner is not the lowest index of its position")
    HX, HY = X[h], Y[h]
    if h.size >= 3:
        nx, ny = np.roll(HX, -1), np.roll(HY, -1)
        px, py = np.roll(HX, 1), np.roll(HY, 1)
        if np.any(_det(px, py, HX, HY, nx, ny) <= 0):
            errs.append("not a strict left turn at every corner")
        for k in range(h.size):
            d = _det(HX[k], HY[k], nx[k], ny[k], X, Y)
            if np.any(d < 0):
                errs.append("an input point lies outside an edge")
                break
    elif h.size == 2:
        d = _det(HX[0], HY[0], HX[1], HY[1], X, Y)
        lo_x, hi_x = min(HX), max(HX)
        lo_y, hi_y = min(HY), max(HY)
        if HX[0] == HX[1] and HY[0] == HY[1]:
            errs.append("two corners at one position")
        if np.any(d != 0) or np.any((X < lo_x) | (X > hi_x) | (Y < lo_y) | (Y > hi_y)):
            errs.append("two corners but points off the segment between them")
    else:
        if np.any((X != HX[0]) | (Y != HY[0])):
            errs.append("single corner but points at other positions")
    return errs
