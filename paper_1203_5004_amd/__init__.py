"""Python binding of the MI355X upper-hood / convex-hull library (libwagener_hull.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/wagener_hull.h.  PyTorch
provides device memory and the current stream.  There is no CPU fallback:
if the library has not been built, every call raises.

    import torch, paper_1203_5004_amd as uh
    idx, cnt = uh.upper_hull(points)          # points: cuda float32 [n, 2]
    idx, cnt = uh.convex_hull(points)         # counter-clockwise hull corners
    plan = uh.upper_hull_plan_create(offsets) # host offsets, len S + 1
    plan.run(points, out_idx, out_counts, stats)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libwagener_hull.so")

UH_OK = 0
UH_ERR_ARG = -1
UH_ERR_ALLOC = -2
UH_ERR_HIP = -3
UH_ERR_CAPTURE = -4
UH_ERR_WORKSPACE = -5
UH_ERR_TOO_LARGE = -6
UH_NOALLOC_MAX_N = 1 << 21
UH_ERR_UNSORTED = -10
UH_ERR_RANGE = -11
UH_ERR_GRID = -12

UH_FLAG_FORCE_FALLBACK = 1
UH_FLAG_NO_VALIDATE = 2
UH_FLAG_GRAPH = 4
UH_FLAG_BOTH_HOODS = 8
UH_FLAG_UNSORTED = 16
UH_FLAG_NO_ELIMINATION = 32
UH_FLAG_CHECK_SIGNS = 64

EXPORTS = (
    "upper_hull_status_string", "upper_hull", "upper_hull_noalloc", "convex_hull",
    "upper_hull_batched",
    "upper_hull_workspace_bytes", "upper_hull_set_workspace",
    "upper_hull_plan_create",
    "upper_hull_plan_run", "upper_hull_plan_destroy", "upper_hull_plan_launches",
    "upper_hull_plan_set_probe", "upper_hull_plan_sorted", "upper_hull_plan_config",
    "upper_hull_plan_blocks", "upper_hull_plan_trace",
    "upper_hull_autotune",
    "upper_hull_read_reference",
    "upper_hull_bridge", "upper_hull_orient",
)


class upper_hull_stats(ctypes.Structure):
    _fields_ = [("orient_evals", ctypes.c_uint64), ("fallbacks", ctypes.c_uint64),
                ("sign_errors", ctypes.c_uint64),
                ("rounds", ctypes.c_int32), ("status", ctypes.c_int32)]


# one upper_hull_stats record = STATS_WORDS int64 words of a torch tensor
STATS_WORDS = ctypes.sizeof(upper_hull_stats) // 8


def new_stats(num, device="cuda"):
    """A zeroed device tensor holding `num` upper_hull_stats records."""
    torch = _torch()
    return torch.zeros((num, STATS_WORDS), dtype=torch.int64, device=device)


def decode_stats(words) -> dict:
    """Fields of stats records copied to the host (int64 array [num, STATS_WORDS])."""
    w = np.ascontiguousarray(np.asarray(words, dtype=np.int64).reshape(-1, STATS_WORDS))
    rec = w.view(np.dtype([("orient_evals", "<u8"), ("fallbacks", "<u8"),
                           ("sign_errors", "<u8"),
                           ("rounds", "<i4"), ("status", "<i4")])).reshape(-1)
    return {k: rec[k].copy() for k in rec.dtype.names}


class upper_hull_config(ctypes.Structure):
    _fields_ = [("strip", ctypes.c_int32), ("fan_in", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


_lib = None


def load_library():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1203_5004_amd.build` "
            "(the library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.upper_hull_status_string.argtypes = [ctypes.c_int]
    lib.upper_hull_status_string.restype = ctypes.c_char_p
    lib.upper_hull.argtypes = [p, i64, p, p, p]
    lib.upper_hull.restype = ctypes.c_int
    lib.upper_hull_noalloc.argtypes = [p, i64, p, p, p]
    lib.upper_hull_noalloc.restype = ctypes.c_int
    lib.convex_hull.argtypes = [p, i64, p, p, p]
    lib.convex_hull.restype = ctypes.c_int
    lib.upper_hull_batched.argtypes = [p, p, i32, p, p, p, p]
    lib.upper_hull_batched.restype = ctypes.c_int
    lib.upper_hull_plan_create.argtypes = [p, i32, p, ctypes.POINTER(p)]
    lib.upper_hull_plan_create.restype = ctypes.c_int
    lib.upper_hull_plan_run.argtypes = [p, p, p, p, p, p]
    lib.upper_hull_plan_run.restype = ctypes.c_int
    lib.upper_hull_plan_destroy.argtypes = [p]
    lib.upper_hull_plan_destroy.restype = None
    lib.upper_hull_plan_launches.argtypes = [p, i32]
    lib.upper_hull_plan_launches.restype = ctypes.c_int
    lib.upper_hull_plan_set_probe.argtypes = [p, p, p]
    lib.upper_hull_plan_set_probe.restype = ctypes.c_int
    lib.upper_hull_autotune.argtypes = [p, p, i32, ctypes.c_uint32, i32, p, p, p]
    lib.upper_hull_autotune.restype = ctypes.c_int
    lib.upper_hull_plan_config.argtypes = [p, p]
    lib.upper_hull_plan_config.restype = ctypes.c_int
    lib.upper_hull_plan_blocks.argtypes = [p, i32, p]
    lib.upper_hull_plan_blocks.restype = ctypes.c_int32
    lib.upper_hull_plan_trace.argtypes = [p, p, i32, p, p, p]
    lib.upper_hull_plan_trace.restype = ctypes.c_int
    lib.upper_hull_plan_sorted.argtypes = [p, ctypes.POINTER(p), ctypes.POINTER(p)]
    lib.upper_hull_plan_sorted.restype = ctypes.c_int
    lib.upper_hull_read_reference.argtypes = [p, i64, i32, p, p]
    lib.upper_hull_read_reference.restype = ctypes.c_int
    lib.upper_hull_workspace_bytes.argtypes = [i64, i32]
    lib.upper_hull_workspace_bytes.restype = ctypes.c_size_t
    lib.upper_hull_set_workspace.argtypes = [p, ctypes.c_size_t]
    lib.upper_hull_set_workspace.restype = ctypes.c_int
    lib.upper_hull_bridge.argtypes = [p, i32, p, i32, i32, p, p]
    lib.upper_hull_bridge.restype = ctypes.c_int
    lib.upper_hull_orient.argtypes = [p, p, p, i64, p, p, i32, p]
    lib.upper_hull_orient.restype = ctypes.c_int
    _lib = lib
    return lib


def upper_hull_status_string(status: int) -> str:
    return load_library().upper_hull_status_string(int(status)).decode()


def _check(rc: int):
    if rc != UH_OK:
        raise RuntimeError(f"upper_hull: {upper_hull_status_string(rc)} ({rc})")


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def upper_hull(points, out_idx=None, out_count=None, stream=None):
    """Upper-hood corner indices of points (cuda float32 [n, 2], x-sorted).

    Returns (out_idx int32[n], out_count int32[1]) on the device; the first
    out_count[0] entries of out_idx are the corners, left to right (a
    negative count is a data-error status).  Asynchronous on `stream`."""
    return _single("upper_hull", points, out_idx, out_count, stream)


def upper_hull_noalloc(points, out_idx=None, out_count=None, stream=None):
    """As ``upper_hull``, in the library's fixed per-device scratch: the call
    allocates no device memory (at most UH_NOALLOC_MAX_N points; calls that
    overlap in time on one device race).  Pass out_idx / out_count to keep
    the call itself free of allocations."""
    return _single("upper_hull_noalloc", points, out_idx, out_count, stream)


def convex_hull(points, out_idx=None, out_count=None, stream=None):
    """Convex-hull corner indices of points (cuda float32 [n, 2], x-sorted),
    counter-clockwise from the lowest point of least x; returned as for
    ``upper_hull``."""
    return _single("convex_hull", points, out_idx, out_count, stream)


def _single(name, points, out_idx, out_count, stream):
    torch = _torch()
    _dev_tensor(points, torch.float32, "points")
    n = points.shape[0]
    if points.dim() != 2 or points.shape[1] != 2:
        raise ValueError("points must have shape [n, 2]")
    if out_idx is None:
        out_idx = torch.empty(max(n, 1), dtype=torch.int32, device=points.device)
    if out_count is None:
        out_count = torch.empty(1, dtype=torch.int32, device=points.device)
    _dev_tensor(out_idx, torch.int32, "out_idx")
    _dev_tensor(out_count, torch.int32, "out_count")
    if out_idx.numel() < n or out_count.numel() < 1:
        raise ValueError("out_idx needs n entries and out_count one")
    _check(getattr(load_library(), name)(_ptr(points), n, _ptr(out_idx), _ptr(out_count),
                                         _stream(stream)))
    return out_idx, out_count


def upper_hull_batched(points, set_offsets, out_idx=None, out_counts=None, stats=None,
                       stream=None):
    """Upper hoods of every set (host offsets, len S + 1) with a cached plan.
    Returns (out_idx int32[N], out_counts int32[S]); set s's corners are at
    out_idx[offsets[s]:offsets[s] + out_counts[s]]."""
    torch = _torch()
    _dev_tensor(points, torch.float32, "points")
    off = np.ascontiguousarray(np.asarray(set_offsets, dtype=np.int64))
    S, N = off.shape[0] - 1, int(off[-1])
    if S < 1 or points.numel() != 2 * N:
        raise ValueError("points do not match set_offsets")
    if out_idx is None:
        out_idx = torch.empty(max(N, 1), dtype=torch.int32, device=points.device)
    if out_counts is None:
        out_counts = torch.empty(S, dtype=torch.int32, device=points.device)
    _dev_tensor(out_idx, torch.int32, "out_idx")
    _dev_tensor(out_counts, torch.int32, "out_counts")
    if out_idx.numel() < N or out_counts.numel() < S:
        raise ValueError("output buffers too small")
    if stats is not None:
        _dev_tensor(stats, torch.int64, "stats")
        if stats.numel() < STATS_WORDS * S:
            raise ValueError(f"stats needs {STATS_WORDS} int64 per set (new_stats)")
    _check(load_library().upper_hull_batched(_ptr(points), off.ctypes.data, S, _ptr(out_idx),
                                             _ptr(out_counts), _ptr(stats), _stream(stream)))
    return out_idx, out_counts


class Plan:
    """A batched plan (schedule + workspace) for fixed set sizes."""

    def __init__(self, set_offsets, strip=0, fan_in=0, flags=0):
        off = np.ascontiguousarray(np.asarray(set_offsets, dtype=np.int64))
        if off.ndim != 1 or off.shape[0] < 2:
            raise ValueError("set_offsets must be 1-D with at least 2 entries")
        self.set_offsets = off
        self.num_sets = off.shape[0] - 1
        self.total = int(off[-1])
        # with both hoods every output array has two halves (upper, lower)
        self.hoods = 2 if flags & UH_FLAG_BOTH_HOODS else 1
        cfg = upper_hull_config(strip, fan_in, flags)
        h = ctypes.c_void_p()
        _check(load_library().upper_hull_plan_create(
            off.ctypes.data, self.num_sets, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    @property
    def config(self) -> dict:
        """The plan's strip, fan_in and flags, defaults resolved."""
        c = upper_hull_config()
        _check(load_library().upper_hull_plan_config(self._h, ctypes.byref(c)))
        return {"strip": c.strip, "fan_in": c.fan_in, "flags": c.flags}

    @property
    def launches(self) -> int:
        """Kernel launches per run without stats."""
        return load_library().upper_hull_plan_launches(self._h, 0)

    def launches_with_stats(self) -> int:
        return load_library().upper_hull_plan_launches(self._h, 1)

    def set_probe(self, before, after):
        """Record raw hipEvent_t handles (ints) around the tile kernel."""
        _check(load_library().upper_hull_plan_set_probe(
            self._h, ctypes.c_void_p(before), ctypes.c_void_p(after)))

    def sorted_view(self):
        """(sorted points, permutation) of the last run of an UH_FLAG_UNSORTED
        plan, copied to the host as numpy arrays (synchronises the device)."""
        torch = _torch()
        sp, pm = ctypes.c_void_p(), ctypes.c_void_p()
        _check(load_library().upper_hull_plan_sorted(self._h, ctypes.byref(sp), ctypes.byref(pm)))
        torch.cuda.synchronize()
        n = self.total
        xy = np.empty((n, 2), np.float32)
        perm = np.empty(n, np.int32)
        if n:
            hip = ctypes.CDLL("libamdhip64.so")
            d2h = 2  # hipMemcpyDeviceToHost
            assert hip.hipMemcpy(ctypes.c_void_p(xy.ctypes.data), sp, ctypes.c_size_t(8 * n), d2h) == 0
            assert hip.hipMemcpy(ctypes.c_void_p(perm.ctypes.data), pm, ctypes.c_size_t(4 * n), d2h) == 0
        return xy, perm

    @property
    def passes(self) -> int:
        """Merge passes of a run (levels of the merge tree above the tiles)."""
        k = 0
        while load_library().upper_hull_plan_blocks(self._h, k + 1, None) >= 0:
            k += 1
        return k

    def blocks(self, level: int) -> np.ndarray:
        """(first point, point count) of every block of a merge-tree level."""
        lib = load_library()
        nb = lib.upper_hull_plan_blocks(self._h, level, None)
        _check(min(nb, 0))
        r = np.zeros((max(nb, 1), 2), dtype=np.int64)
        _check(min(lib.upper_hull_plan_blocks(self._h, level, r.ctypes.data), 0))
        return r[:nb]

    def trace(self, points, level: int, stream=None):
        """Run up to a merge-tree level and return, on the host, every block's
        (count, corner indices relative to its set); see upper_hull_plan_trace."""
        torch = _torch()
        _dev_tensor(points, torch.float32, "points")
        rng = self.blocks(level)
        out = torch.full((max(self.hoods * self.total, 1),), -7, dtype=torch.int32,
                         device=points.device)
        cnt = torch.full((max(len(rng), 1),), -7, dtype=torch.int32, device=points.device)
        _check(load_library().upper_hull_plan_trace(self._h, _ptr(points), level, _ptr(out),
                                                    _ptr(cnt), _stream(stream)))
        torch.cuda.synchronize()
        o, c = out.cpu().numpy(), cnt.cpu().numpy()
        res = []
        for b, (s, _) in enumerate(rng):
            raw = int(c[b])
            if -1000 < raw < 0:  # a data-error status
                res.append((raw, None))
            else:
                res.append((raw, o[s:s + (raw & 0x7fffffff)].copy()))
        return res

    def run(self, points, out_idx, out_counts, stats=None, stream=None):
        torch = _torch()
        _dev_tensor(points, torch.float32, "points")
        _dev_tensor(out_idx, torch.int32, "out_idx")
        _dev_tensor(out_counts, torch.int32, "out_counts")
        if points.numel() != 2 * self.total or out_idx.numel() < self.hoods * self.total:
            raise ValueError("buffer sizes do not match the plan")
        if out_counts.numel() < self.hoods * self.num_sets:
            raise ValueError("out_counts too small")
        if stats is not None:
            _dev_tensor(stats, torch.int64, "stats")
            if stats.numel() < STATS_WORDS * self.hoods * self.num_sets:
                raise ValueError("stats needs one record per set and hood (new_stats)")
        _check(load_library().upper_hull_plan_run(
            self._h, _ptr(points), _ptr(out_idx), _ptr(out_counts), _ptr(stats),
            _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().upper_hull_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upper_hull_plan_create(set_offsets, strip=0, fan_in=0, flags=0) -> Plan:
    return Plan(set_offsets, strip, fan_in, flags)


def upper_hull_autotune(points, set_offsets, flags=0, reps=3, stream=None):
    """Time the candidate (strip, fan_in) pairs on `points` (cuda float32
    [N, 2]) for this set layout; returns (config dict, mean ms per run)."""
    torch = _torch()
    _dev_tensor(points, torch.float32, "points")
    off = np.ascontiguousarray(np.asarray(set_offsets, dtype=np.int64))
    if off.ndim != 1 or off.shape[0] < 2 or points.numel() != 2 * int(off[-1]):
        raise ValueError("points do not match set_offsets")
    best = upper_hull_config()
    ms = ctypes.c_float()
    _check(load_library().upper_hull_autotune(_ptr(points), off.ctypes.data, off.shape[0] - 1,
                                              flags, reps, ctypes.byref(best),
                                              ctypes.byref(ms), _stream(stream)))
    return {"strip": best.strip, "fan_in": best.fan_in, "flags": best.flags}, ms.value


def upper_hull_read_reference(points, reps=20, stream=None):
    """Mean ms of a plain streaming read of `points` (cuda float32 [N, 2])."""
    torch = _torch()
    _dev_tensor(points, torch.float32, "points")
    ms = ctypes.c_float()
    _check(load_library().upper_hull_read_reference(_ptr(points), points.numel() // 2, reps,
                                                    ctypes.byref(ms), _stream(stream)))
    return ms.value


def upper_hull_workspace_bytes(max_total_n: int, max_sets: int = 1) -> int:
    """Bytes of a workspace that serves every single-set call with at most
    max_total_n points over max_sets sets (convex_hull of n points: 2 n points
    over 2 sets)."""
    return int(load_library().upper_hull_workspace_bytes(int(max_total_n), int(max_sets)))


def upper_hull_set_workspace(buffer):
    """Let the single-set calls on the buffer's device use `buffer` (a CUDA
    uint8 tensor, 256-byte aligned; keep it alive while it is set), or go back
    to library memory with None.  Returns the buffer."""
    torch = _torch()
    if buffer is None:
        _check(load_library().upper_hull_set_workspace(ctypes.c_void_p(0), 0))
        return None
    _dev_tensor(buffer, torch.uint8, "buffer")
    _check(load_library().upper_hull_set_workspace(_ptr(buffer), buffer.numel()))
    return buffer


def upper_hull_bridge(P, Q, lanes=64, stream=None):
    """Bridge (a, b) of two hoods given as cuda float32 [h, 2] corner lists."""
    torch = _torch()
    _dev_tensor(P, torch.float32, "P")
    _dev_tensor(Q, torch.float32, "Q")
    out = torch.empty(2, dtype=torch.int32, device=P.device)
    _check(load_library().upper_hull_bridge(_ptr(P), P.shape[0], _ptr(Q), Q.shape[0],
                                            lanes, _ptr(out), _stream(stream)))
    return out


def upper_hull_orient(a, b, c, force_fallback=False, stream=None):
    """Exact orientation signs (int8) and fallback flags (uint8) per row."""
    torch = _torch()
    for t, nm in ((a, "a"), (b, "b"), (c, "c")):
        _dev_tensor(t, torch.float32, nm)
    m = a.shape[0]
    sign = torch.empty(max(m, 1), dtype=torch.int8, device=a.device)
    fb = torch.empty(max(m, 1), dtype=torch.uint8, device=a.device)
    _check(load_library().upper_hull_orient(_ptr(a), _ptr(b), _ptr(c), m, _ptr(sign),
                                            _ptr(fb), int(bool(force_fallback)),
                                            _stream(stream)))
    return sign[:m], fb[:m]
