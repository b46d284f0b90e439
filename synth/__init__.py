"""Seeded synthetic point sets for the upper-hull workloads.

This module is shared by the CPU oracle's tests and by the GPU path's tests
and benchmark.  It only *draws inputs*: it holds none of the hull method's
arithmetic (no orientation test, no hull, no merge).  Every array it returns
is float32, shape (n, 2), x non-decreasing, with both coordinates on a dyadic
grid (multiples of 2**-G), so the exact-integer oracle and the GPU predicate
can both treat them exactly.

Recipes (integer-first, then scaled by 2**-G exactly, numpy PCG64):

* ``uniform(n, G)``    x = sorted distinct k in [0, 2**G) drawn without
                       replacement, y = m * 2**-G with m ~ U{0 .. 2**G - 1}.
* ``uniform_iid(n, G)``  x = sorted iid k ~ U{0 .. 2**G - 1} (equal x occur),
                       rounded to float32 (RNE) -- for G > 24 this coarsens
                       x (and y) in [2**(24-G), 1), which creates long equal-x
                       runs; the result is still on the 2**-G grid.
* ``arc(n, G, jitter)`` x = sorted distinct k, y = round(sqrt(X (2**G - X)))
                       + U{-jitter .. jitter} in grid units (a semicircle of
                       radius 1/2 plus jitter: a large hull).
* ``parabola(n, G, jitter)`` x = sorted distinct k, Y = RNE(X (2**G - X) / 2**G)
                       + U{-jitter .. jitter} (y = x - x^2 snapped to the grid:
                       many near-collinear and exactly collinear triples).
* ``batched_mixed``    4096 sets, sizes floor(2**(6 + 14 u)), powers of two
                       bumped by one; even sets uniform, odd sets arc (jitter
                       4), G = 20.
* ``batched_parabola`` 1024 sets of 2**18 points, parabola with jitter 1,
                       G = 20.

The five named workloads (``WORKLOADS``) follow the configurations the
benchmark and the parity tests use; each takes an optional size override so
tests can draw the same recipe at a size the oracle finishes in seconds.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 12035004


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _to_f32(ints: np.ndarray, G: int) -> np.ndarray:
    """Integer grid coordinates -> float32 (exact when |k| < 2**24, else RNE)."""
    return (ints.astype(np.float64) * (2.0 ** -G)).astype(np.float32)


def _pack(X: np.ndarray, Y: np.ndarray, G: int) -> np.ndarray:
    out = np.empty((X.shape[0], 2), dtype=np.float32)
    out[:, 0] = _to_f32(X, G)
    out[:, 1] = _to_f32(Y, G)
    return out


def _distinct_sorted(rng: np.random.Generator, n: int, G: int) -> np.ndarray:
    N = 1 << G
    if n > N:
        raise ValueError(f"cannot draw {n} distinct x on a 2**-{G} grid")
    if n == N:
        return np.arange(N, dtype=np.int64)
    k = rng.choice(N, size=n, replace=False, shuffle=False)
    k = np.asarray(k, dtype=np.int64)
    k.sort()
    return k


def _isqrt_round(v: np.ndarray) -> np.ndarray:
    """round(sqrt(v)) for non-negative int64 v < 2**52, computed exactly."""
    r = np.floor(np.sqrt(v.astype(np.float64))).astype(np.int64)
    r -= (r * r > v).astype(np.int64)
    r += ((r + 1) * (r + 1) <= v).astype(np.int64)
    # round half: v >= r^2 + r + 1  <=>  sqrt(v) > r + 1/2
    r += (v - r * r > r).astype(np.int64)
    return r


def uniform(n: int, G: int = 20, seed: int = SEED_BASE) -> np.ndarray:
    rng = _rng(seed)
    X = _distinct_sorted(rng, n, G)
    Y = rng.integers(0, 1 << G, size=n, dtype=np.int64)
    return _pack(X, Y, G)


def uniform_iid(n: int, G: int = 27, seed: int = SEED_BASE) -> np.ndarray:
    rng = _rng(seed)
    X = rng.integers(0, 1 << G, size=n, dtype=np.int64)
    X.sort()
    Y = rng.integers(0, 1 << G, size=n, dtype=np.int64)
    return _pack(X, Y, G)


def arc(n: int, G: int = 24, jitter: int = 4, seed: int = SEED_BASE) -> np.ndarray:
    rng = _rng(seed)
    X = _distinct_sorted(rng, n, G)
    Y = _isqrt_round(X * ((1 << G) - X))
    Y += rng.integers(-jitter, jitter + 1, size=n, dtype=np.int64)
    return _pack(X, Y, G)


def parabola(n: int, G: int = 20, jitter: int = 1, seed: int = SEED_BASE) -> np.ndarray:
    rng = _rng(seed)
    X = _distinct_sorted(rng, n, G)
    num = X * ((1 << G) - X)
    q, r = np.divmod(num, 1 << G)
    half = 1 << (G - 1)
    # round half to even
    Y = q + ((r > half) | ((r == half) & (q % 2 == 1))).astype(np.int64)
    Y += rng.integers(-jitter, jitter + 1, size=n, dtype=np.int64)
    return _pack(X, Y, G)


def log_uniform_sizes(num_sets: int, lo_log2: int, hi_log2: int, seed: int) -> np.ndarray:
    rng = _rng(seed)
    u = rng.random(num_sets)
    s = np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    pow2 = (s & (s - 1)) == 0
    s[pow2] += 1
    return s


def concat_sets(sets: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    sizes = np.array([s.shape[0] for s in sets], dtype=np.int64)
    offsets = np.zeros(len(sets) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pts = np.concatenate(sets, axis=0) if sets else np.zeros((0, 2), np.float32)
    return np.ascontiguousarray(pts, dtype=np.float32), offsets


def batched_mixed(num_sets: int = 4096, lo_log2: int = 6, hi_log2: int = 20,
                  G: int = 20, seed: int = SEED_BASE + 3):
    sizes = log_uniform_sizes(num_sets, lo_log2, hi_log2, seed)
    sizes = np.minimum(sizes, 1 << G)
    sets = []
    for s, n in enumerate(sizes):
        if s % 2 == 0:
            sets.append(uniform(int(n), G, seed=seed * 7919 + s))
        else:
            sets.append(arc(int(n), G, 4, seed=seed * 7919 + s))
    return concat_sets(sets)


def batched_parabola(num_sets: int = 1024, set_size: int = 1 << 18, G: int = 20,
                     seed: int = SEED_BASE + 4):
    sets = [parabola(set_size, G, 1, seed=seed * 7919 + s) for s in range(num_sets)]
    return concat_sets(sets)


def _single(pts: np.ndarray):
    return pts, np.array([0, pts.shape[0]], dtype=np.int64)


# name -> (builder(size_override or None) -> (points, offsets), description)
WORKLOADS = {
    "uniform_2^16": (
        lambda n=None: _single(uniform(n or (1 << 16), 20, SEED_BASE + 0)),
        "1 set, n=2^16, distinct x on the 2^-20 grid, y uniform on the 2^-20 grid"),
    "arc_2^24": (
        lambda n=None: _single(arc(n or (1 << 24), 24, 4, SEED_BASE + 1)),
        "1 set, n=2^24, x = every 2^-24 grid point, y = semicircle + U{-4..4} units"),
    "uniform_2^27": (
        lambda n=None: _single(uniform_iid(n or (1 << 27), 27, SEED_BASE + 2)),
        "1 set, n=2^27, x iid on the 2^-27 grid (sorted, float32 RNE), y uniform"),
    "batched_mixed_4096": (
        lambda n=None: batched_mixed(n or 4096),
        "4096 sets, sizes log-uniform in [2^6, 2^20] (no powers of two), "
        "half uniform, half arc, 2^-20 grid"),
    "batched_parabola_1024x2^18": (
        lambda n=None: batched_parabola(n or 1024),
        "1024 sets x 2^18, y = x - x^2 snapped to the 2^-20 grid + U{-1,0,1}"),
}


# ---------------------------------------------------------------- tiny sets
def lattice_points(n: int, side: int, seed: int, allow_dup: bool = True) -> np.ndarray:
    """n points with integer coordinates in [0, side) x [0, side), scaled by
    1/side (side a power of two), sorted by x (stable), duplicates allowed."""
    rng = _rng(seed)
    G = int(side).bit_length() - 1
    assert 1 << G == side
    X = rng.integers(0, side, size=n, dtype=np.int64)
    Y = rng.integers(0, side, size=n, dtype=np.int64)
    if not allow_dup:
        key = X * side + Y
        _, first = np.unique(key, return_index=True)
        X, Y = X[np.sort(first)], Y[np.sort(first)]
    order = np.argsort(X, kind="stable")
    return _pack(X[order], Y[order], G)


def from_integers(X, Y, G: int) -> np.ndarray:
    X = np.asarray(X, dtype=np.int64)
    Y = np.asarray(Y, dtype=np.int64)
    return _pack(X, Y, G)
