"""CPU oracle for the upper and lower hoods and the convex hull -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never loads it and shares no
code with it; the two meet only through the seeded generators in ``synth``.

Contents:
  * ``hull_oracle.c`` (built into ``_build/liboracle_hull.so``): the exact
    integer Andrew monotone chain (upper half) -- the plain definition of the
    upper hood the method computes -- the lower hood as its mirror image, and
    the convex hull assembled from both (counter-clockwise);
  * ``brute``      -- O(n^3) evaluation of the hood's definition (tiny n);
  * ``invariants`` -- exact checks that characterise the strict upper hood;
  * ``bridge``     -- the per-merge quantities of the paper's match-and-merge
    step (tangent classifiers g and f, the common tangent) by brute force;
  * ``unsorted_hull`` -- any of the three for points in any order: a stable
    sort by x in front (a library sort as one step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hull_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle_hull.so")

# status codes (the oracle's own copy of the documented contract values)
OK = 0
ERR_ARG = -1
ERR_UNSORTED = -10
ERR_RANGE = -11
ERR_GRID = -12

_lib = None


def _compile(out: str, extra: list[str]) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", *extra, "-std=gnu11", "-shared", "-fPIC",
                           "-Wall", "-Werror", _SRC, "-o", tmp, "-lm", "-lpthread"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/_build/liboracle_hull.so
    (portable code: the library also runs on other hosts)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        _compile(_LIB_PATH, [])
    return _LIB_PATH


def build_native(directory: str) -> str:
    """Compile the oracle with -O3 -march=native for the CPU this runs on, into
    `directory` (for the CPU baseline's timing; a library built for one CPU
    may not run on another, so it is built where it is timed)."""
    os.makedirs(directory, exist_ok=True)
    out = os.path.join(directory, "liboracle_hull_native.so")
    _compile(out, ["-march=native"])
    return out


def _declare(lib):
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_upper_hull.argtypes = [p, i64, p, p]
    lib.oracle_upper_hull.restype = ctypes.c_int
    lib.oracle_upper_hull_batched.argtypes = [p, p, i64, p, p]
    lib.oracle_upper_hull_batched.restype = ctypes.c_int
    for name in ("oracle_lower_hull", "oracle_convex_hull"):
        getattr(lib, name).argtypes = [p, i64, p, p]
        getattr(lib, name).restype = ctypes.c_int
    lib.oracle_lower_hull_batched.argtypes = [p, p, i64, p, p]
    lib.oracle_lower_hull_batched.restype = ctypes.c_int
    lib.oracle_orient_signs.argtypes = [p, p, p, i64, p]
    lib.oracle_orient_signs.restype = ctypes.c_int
    lib.oracle_hood_mt.argtypes = [p, i64, i32, i32, p, p]
    lib.oracle_hood_mt.restype = ctypes.c_int
    lib.oracle_hood_batched_mt.argtypes = [p, p, i64, i32, i32, p, p]
    lib.oracle_hood_batched_mt.restype = ctypes.c_int
    lib.oracle_online_cpus.argtypes = []
    lib.oracle_online_cpus.restype = ctypes.c_int32
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def load_native(directory: str):
    """The -march=native build (see build_native), loaded separately from the
    portable one; it exposes the same functions."""
    return _declare(ctypes.CDLL(build_native(directory)))


def _pts(xy) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.float32).reshape(-1, 2))
    return a


def _single(name, xy):
    a = _pts(xy)
    n = a.shape[0]
    out = np.empty(max(n, 1), dtype=np.int32)
    cnt = ctypes.c_int64(0)
    rc = getattr(_load(), name)(a.ctypes.data, n, out.ctypes.data, ctypes.addressof(cnt))
    return rc, out[: cnt.value].copy()


def upper_hull_status(xy):
    """(status, indices).  status 0 on success, else a negative error code."""
    return _single("oracle_upper_hull", xy)


def lower_hull_status(xy):
    """(status, indices) of the lower hood (corners left to right)."""
    return _single("oracle_lower_hull", xy)


def convex_hull_status(xy):
    """(status, indices) of the convex hull, counter-clockwise from the lowest
    point of least x."""
    return _single("oracle_convex_hull", xy)


def upper_hull(xy) -> np.ndarray:
    """Indices of the strict upper-hood corners, left to right (int32)."""
    rc, idx = upper_hull_status(xy)
    if rc != OK:
        raise ValueError(f"oracle: invalid input (status {rc})")
    return idx


def lower_hull(xy) -> np.ndarray:
    """Indices of the strict lower-hood corners, left to right (int32)."""
    rc, idx = lower_hull_status(xy)
    if rc != OK:
        raise ValueError(f"oracle: invalid input (status {rc})")
    return idx


def convex_hull(xy) -> np.ndarray:
    """Indices of the convex hull's corners, counter-clockwise (int32)."""
    rc, idx = convex_hull_status(xy)
    if rc != OK:
        raise ValueError(f"oracle: invalid input (status {rc})")
    return idx


def _batched(name, xy, offsets, lib=None):
    a = _pts(xy)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    S = off.shape[0] - 1
    out = np.zeros(max(a.shape[0], 1), dtype=np.int32)
    counts = np.zeros(max(S, 1), dtype=np.int64)
    rc = getattr(_lib_or(lib), name)(a.ctypes.data, off.ctypes.data, S,
                                     out.ctypes.data, counts.ctypes.data)
    if rc != OK:
        raise ValueError(f"oracle: invalid input (status {rc})")
    return out, counts[:S]


def upper_hull_batched(xy, offsets, lib=None):
    """Per-set hulls.  Returns (out_idx, counts): set s's corner indices,
    relative to offsets[s], are out_idx[offsets[s] : offsets[s] + counts[s]].
    `lib`: another build of the same source (``load_native``)."""
    return _batched("oracle_upper_hull_batched", xy, offsets, lib)


def lower_hull_batched(xy, offsets, lib=None):
    """Per-set lower hoods, laid out as in ``upper_hull_batched``."""
    return _batched("oracle_lower_hull_batched", xy, offsets, lib)


def orient_signs(a, b, c) -> np.ndarray:
    """Exact sign of det(b - a, c - a) for each row (int8 in {-1, 0, 1})."""
    a, b, c = _pts(a), _pts(b), _pts(c)
    m = a.shape[0]
    assert b.shape[0] == m and c.shape[0] == m
    out = np.empty(max(m, 1), dtype=np.int8)
    rc = _load().oracle_orient_signs(a.ctypes.data, b.ctypes.data,
                                     c.ctypes.data, m, out.ctypes.data)
    if rc != OK:
        raise ValueError(f"oracle: invalid coordinate (status {rc})")
    return out[:m].copy()

def sort_order(xy) -> np.ndarray:
    """The order in which the hull of points given in any order is taken:
    stable by x (equal x keep their input order, so every tie rule that
    prefers the lowest index still prefers the lowest input index).  -0.0
    and +0.0 compare equal."""
    a = _pts(xy)
    return np.argsort(a[:, 0], kind="stable").astype(np.int64)


def unsorted_hull(xy, hood: str = "upper"):
    """(status, indices) of the upper hood, lower hood or convex hull of
    points in any order: the hull of the points sorted by ``sort_order``,
    its corners mapped back to input indices (corners left to right; the
    convex hull counter-clockwise)."""
    a = _pts(xy)
    order = sort_order(a)
    fn = {"upper": upper_hull_status, "lower": lower_hull_status,
          "convex": convex_hull_status}[hood]
    rc, idx = fn(a[order])
    return rc, order[idx].astype(np.int32)


def _lib_or(lib):
    return lib if lib is not None else _load()


def hood_mt(xy, threads: int, lower: bool = False, lib=None):
    """(status, indices) of the upper (or lower) hood computed on `threads`
    threads: chunks cut at equal-x run boundaries, a chain per chunk, then one
    chain over the chunk hoods.  Same result and status as the single chain."""
    a = _pts(xy)
    n = a.shape[0]
    out = np.empty(max(n, 1), dtype=np.int32)
    cnt = ctypes.c_int64(0)
    rc = _lib_or(lib).oracle_hood_mt(a.ctypes.data, n, int(threads), int(bool(lower)),
                                     out.ctypes.data, ctypes.addressof(cnt))
    return rc, out[: cnt.value].copy()


def hood_batched_mt(xy, offsets, threads: int, lower: bool = False, lib=None):
    """Per-set hoods on `threads` threads (sets taken in order as threads become
    free); (status, out_idx, counts) laid out as ``upper_hull_batched``."""
    a = _pts(xy)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    S = off.shape[0] - 1
    out = np.zeros(max(a.shape[0], 1), dtype=np.int32)
    counts = np.zeros(max(S, 1), dtype=np.int64)
    rc = _lib_or(lib).oracle_hood_batched_mt(a.ctypes.data, off.ctypes.data, S, int(threads),
                                             int(bool(lower)), out.ctypes.data,
                                             counts.ctypes.data)
    return rc, out, counts[:S]


def online_cpus() -> int:
    return int(_load().oracle_online_cpus())
