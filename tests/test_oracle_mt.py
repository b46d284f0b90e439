"""Pins for the oracle's all-cores variants (used only to time the CPU
baseline): they must return exactly what the single chain returns -- same
corners, same data-error status -- for every thread count, including chunk
cuts that fall inside runs of equal x (moved to the run's start) and errors
near chunk boundaries.  Tiny inputs are also checked against brute force of
the hood's definition directly.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import brute

THREADS = (1, 2, 3, 7, 16, 64)


def _recipes():
    yield "uniform", synth.uniform(5000, 20, seed=11)
    yield "uniform_iid", synth.uniform_iid(20000, 27, seed=12)   # equal-x runs
    yield "arc", synth.arc(6000, 20, 4, seed=13)                  # large hood
    yield "parabola", synth.parabola(6000, 20, 1, seed=14)        # collinear triples


@pytest.mark.parametrize("name,xy", list(_recipes()), ids=lambda v: v if isinstance(v, str) else "")
@pytest.mark.parametrize("lower", [False, True])
def test_equals_single_chain(name, xy, lower):
    ref_rc, ref = (oracle.lower_hull_status if lower else oracle.upper_hull_status)(xy)
    assert ref_rc == 0
    for t in THREADS:
        rc, got = oracle.hood_mt(xy, t, lower=lower)
        assert rc == 0 and np.array_equal(got, ref), (name, t)


def test_runs_of_equal_x_cut_across_chunks():
    # 12 distinct x, runs of 1 .. 300 points: nominal cuts fall inside runs;
    # the highest point of a run sits at its start, middle or end, and some
    # runs hold ties (the lowest index must win)
    rng = np.random.default_rng(3)
    X, Y = [], []
    for k, run in enumerate([1, 300, 7, 250, 2, 131, 299, 5, 64, 200, 3, 90]):
        ys = rng.integers(0, 40, size=run)
        where = k % 3
        top = 60 + (k * 7) % 11
        ys[0 if where == 0 else (run // 2 if where == 1 else run - 1)] = top
        if run > 3 and k % 2:
            ys[run // 3] = top  # a tie with the highest point
        X += [k * 5] * run
        Y += list(ys)
    xy = synth.from_integers(np.array(X), np.array(Y), 8)
    ref = oracle.upper_hull(xy)
    for t in list(THREADS) + [5, 11, 13, 1000, 1024]:
        for lower in (False, True):
            rc, got = oracle.hood_mt(xy, t, lower=lower)
            want = oracle.lower_hull(xy) if lower else ref
            assert rc == 0 and np.array_equal(got, want), (t, lower)


def test_brute_force_on_tiny_lattices():
    for seed in range(60):
        n = 1 + seed % 9
        xy = synth.lattice_points(n, 4, seed=seed)
        want = brute.upper_hull_brute(xy)
        for t in (1, 2, 3, 4, 8):
            rc, got = oracle.hood_mt(xy, t)
            assert rc == 0 and list(got) == want, (seed, t)


def test_empty_and_tiny():
    for t in (1, 4):
        assert oracle.hood_mt(np.zeros((0, 2), np.float32), t)[1].size == 0
        assert list(oracle.hood_mt([[0.5, 0.5]], t)[1]) == [0]
        assert list(oracle.hood_mt([[0.25, 0.5], [0.75, 0.5]], t)[1]) == [0, 1]


@pytest.mark.parametrize("kind", ["x_range", "y_grid", "unsorted", "nan", "neg_x"])
def test_error_status_equals_single_chain(kind):
    base = synth.uniform(4096, 20, seed=21)
    for pos in (0, 1, 511, 512, 513, 1023, 1024, 2047, 4095):
        for second in (None, 3000, 100):
            xy = base.copy()
            for p in [pos] + ([second] if second is not None else []):
                if kind == "x_range":
                    xy[p, 0] = 1.5
                elif kind == "y_grid":
                    xy[p, 1] = np.float32(3 * 2 ** -31)  # not a multiple of 2^-30
                elif kind == "unsorted":
                    xy[p, 0] = xy[p - 1, 0] - np.float32(2 ** -20) if p > 0 else xy[p, 0]
                    if p == 0:
                        xy[1, 0] = np.float32(0.0)
                        xy[0, 0] = np.float32(2 ** -10)
                elif kind == "nan":
                    xy[p, 1] = np.nan
                else:
                    xy[p, 0] = np.float32(-2 ** -30)
            ref_rc, _ = oracle.upper_hull_status(xy)
            assert ref_rc < 0
            for t in (2, 4, 8, 64):
                rc, _ = oracle.hood_mt(xy, t)
                assert rc == ref_rc, (kind, pos, second, t)


def _batched_single(pts, off, lower):
    """The single-thread batched oracle with per-set statuses (it does not stop
    at the first failing set)."""
    lib = oracle._load()
    a = np.ascontiguousarray(pts)
    o = np.ascontiguousarray(off)
    S = len(off) - 1
    out = np.zeros(len(a), np.int32)
    cnt = np.zeros(S, np.int64)
    fn = lib.oracle_lower_hull_batched if lower else lib.oracle_upper_hull_batched
    rc = fn(a.ctypes.data, o.ctypes.data, S, out.ctypes.data, cnt.ctypes.data)
    return rc, out, cnt


def test_batched_equals_single_thread():
    pts, off = synth.batched_mixed(64)
    pts = pts.copy()
    for s in (3, 17, 40):  # data errors in a few sets: each reports its own status
        a = int(off[s])
        pts[a + (int(off[s + 1]) - a) // 2, 1] = 2.0
    for lower in (False, True):
        rc1, out1, cnt1 = _batched_single(pts, off, lower)
        assert rc1 < 0
        for t in (1, 3, 8, 33):
            rc, out, cnt = oracle.hood_batched_mt(pts, off, t, lower=lower)
            assert rc == rc1
            assert np.array_equal(cnt, cnt1)
            for s in range(len(off) - 1):
                c = int(cnt[s])
                if c > 0:
                    assert np.array_equal(out[off[s]:off[s] + c], out1[off[s]:off[s] + c])


def test_online_cpus_is_positive():
    assert oracle.online_cpus() >= 1
