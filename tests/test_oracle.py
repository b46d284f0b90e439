"""Pins for the CPU oracle: values fixed by the paper's definitions and by
mathematics, not by the oracle itself.

* hand-derived fixtures (tests/golden), each citing its passage;
* closed forms (empty, single point, collinear, convex, concave, equal x);
* O(n^3) brute force of the hood's definition on exhaustive and random tiny
  lattices (duplicates, equal-x runs, collinear triples);
* Qhull (scipy) on points in general position -- an independent library;
* exact invariants on the workload recipes at reduced size;
* the contract's error codes.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import brute, invariants
from tests import golden_io


def hull(xy):
    return list(oracle.upper_hull(np.asarray(xy, np.float32)))


# ------------------------------------------------------------------ fixtures
@pytest.mark.parametrize("path", golden_io.all_fixtures(), ids=lambda p: p.split("/")[-1])
def test_golden_fixture(path):
    xy, expect = golden_io.load(path)
    assert hull(xy) == list(expect)
    assert brute.upper_hull_brute(xy) == list(expect)


# -------------------------------------------------------------- closed forms
def test_empty_and_single():
    assert hull(np.zeros((0, 2))) == []
    assert hull([[0.5, 0.25]]) == [0]


def test_two_points():
    assert hull([[0.0, 0.0], [1.0, 0.0]]) == [0, 1]
    assert hull([[0.25, 0.75], [0.5, -0.5]]) == [0, 1]


def test_equal_x_pair_and_duplicates():
    assert hull([[0.5, 0.0], [0.5, 0.25]]) == [1]
    assert hull([[0.5, 0.25], [0.5, 0.0]]) == [0]
    assert hull([[0.5, 0.25], [0.5, 0.25], [0.5, 0.25]]) == [0]


def test_all_collinear_and_constant():
    n = 37
    X = np.arange(n)
    assert hull(synth.from_integers(X, X, 6)) == [0, n - 1]
    assert hull(synth.from_integers(X, np.full(n, 5), 6)) == [0, n - 1]
    assert hull(synth.from_integers(X, 63 - X, 6)) == [0, n - 1]


def test_convex_sequence_keeps_only_ends():
    n = 200
    X = np.arange(n)
    Y = X * X  # strictly convex: every interior point is below the chord
    assert hull(synth.from_integers(X, Y, 16)) == [0, n - 1]


def test_concave_sequence_keeps_all():
    n = 500
    K = 1 << 10
    X = np.arange(n) * 2
    Y = X * (K - X)  # strictly concave (integer, not rounded)
    assert hull(synth.from_integers(X, Y, 20)) == list(range(n))


def test_vertical_stack_only():
    Y = np.array([3, 9, 1, 9, 4])
    assert hull(synth.from_integers(np.zeros(5, np.int64), Y, 4)) == [1]


# --------------------------------------------------------------- brute force
def _lattice_cases():
    pts = [(x, y) for x in range(3) for y in range(3)]
    seen = set()
    for n in range(1, 6):
        for combo in itertools.product(pts, repeat=n):
            seq = tuple(sorted(combo, key=lambda p: p[0]))  # stable: keeps order of equal x
            if seq in seen:
                continue
            seen.add(seq)
            yield seq


def test_brute_force_exhaustive_3x3_up_to_5_points():
    count = 0
    for seq in _lattice_cases():
        X = [p[0] for p in seq]
        Y = [p[1] for p in seq]
        xy = synth.from_integers(X, Y, 2)
        assert hull(xy) == brute.upper_hull_brute(xy), seq
        count += 1
    assert count > 5000


@pytest.mark.parametrize("side", [4, 8, 16])
def test_brute_force_random_lattices(side):
    for seed in range(300):
        n = 1 + seed % 14
        xy = synth.lattice_points(n, side, seed=seed * 31 + side)
        got = hull(xy)
        assert got == brute.upper_hull_brute(xy), (side, seed)
        assert invariants.check(xy, got) == []


def test_brute_force_medium_random():
    for seed in range(20):
        xy = synth.lattice_points(40, 64, seed=1000 + seed)
        assert hull(xy) == brute.upper_hull_brute(xy)


# --------------------------------------------------------------- Qhull check
def _qhull_upper(xy):
    from scipy.spatial import ConvexHull
    h = ConvexHull(xy.astype(np.float64))
    v = list(h.vertices)  # counter-clockwise
    ileft = min(v, key=lambda i: xy[i, 0])
    iright = max(v, key=lambda i: xy[i, 0])
    # counter-clockwise from the rightmost vertex walks the upper chain to the left
    k = v.index(iright)
    chain = []
    while True:
        chain.append(v[k])
        if v[k] == ileft:
            break
        k = (k + 1) % len(v)
    return sorted(chain)


@pytest.mark.parametrize("seed", range(6))
def test_qhull_general_position(seed):
    pytest.importorskip("scipy.spatial")
    rng = np.random.default_rng(seed)
    n = 3000
    X = np.sort(rng.choice(1 << 20, n, replace=False))
    Y = rng.integers(0, 1 << 20, n)
    xy = synth.from_integers(X, Y, 20)
    assert hull(xy) == _qhull_upper(xy)


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("name,n", [("uniform_2^16", 1 << 14), ("arc_2^24", 1 << 14),
                                    ("uniform_2^27", 1 << 16)])
def test_invariants_on_workload_recipes(name, n):
    xy, _ = synth.WORKLOADS[name][0](n)
    h = hull(xy)
    assert invariants.check(xy, h) == []
    assert len(h) >= 2


def test_invariants_parabola_and_arc_recipes():
    for xy in (synth.parabola(1 << 12, 20, 1, seed=5), synth.arc(1 << 12, 20, 4, seed=6)):
        h = hull(xy)
        assert invariants.check(xy, h) == []


def test_invariants_reject_wrong_answers():
    xy = synth.arc(2000, 20, 4, seed=7)
    h = hull(xy)
    assert invariants.check(xy, h) == []
    assert invariants.check(xy, h[:-1]) != []               # dropped end corner
    assert invariants.check(xy, h[:3] + h[4:]) != []         # dropped middle corner
    mid = (h[3] + h[4]) // 2
    assert invariants.check(xy, sorted(h + [mid])) != []     # extra point


# --------------------------------------------------------------- batched
def test_batched_equals_per_set():
    pts, off = synth.batched_mixed(num_sets=24, lo_log2=0, hi_log2=10, seed=99)
    out, counts = oracle.upper_hull_batched(pts, off)
    for s in range(24):
        seg = pts[off[s]:off[s + 1]]
        assert list(out[off[s]:off[s] + counts[s]]) == hull(seg)


# --------------------------------------------------------------- contract
def test_error_codes():
    rc, _ = oracle.upper_hull_status([[0.5, 0.0], [0.25, 0.0]])
    assert rc == oracle.ERR_UNSORTED
    rc, _ = oracle.upper_hull_status([[1.5, 0.0]])
    assert rc == oracle.ERR_RANGE
    rc, _ = oracle.upper_hull_status([[0.5, 1.5]])
    assert rc == oracle.ERR_RANGE
    rc, _ = oracle.upper_hull_status([[float("nan"), 0.0]])
    assert rc == oracle.ERR_RANGE
    rc, _ = oracle.upper_hull_status([[0.5, 2.0 ** -40]])
    assert rc == oracle.ERR_GRID
    rc, _ = oracle.upper_hull_status([[0.0, -1.0], [1.0, 1.0]])
    assert rc == oracle.OK


def test_orient_signs_closed_forms():
    a = np.array([[0, 0], [0, 0], [0, 0], [0.25, 0.5]], np.float32)
    b = np.array([[1, 0], [1, 0], [1, 0], [0.75, 0.5]], np.float32)
    c = np.array([[0.5, 0.5], [0.5, -0.5], [0.5, 0.0], [0.5, 0.5]], np.float32)
    assert list(oracle.orient_signs(a, b, c)) == [1, -1, 0, 0]
