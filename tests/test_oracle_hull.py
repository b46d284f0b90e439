"""Pins of the oracle's lower hood and convex hull (CPU only).

The lower hood is the mirror image of the upper hood under y -> -y; the
convex hull is the lower hood left to right followed by the upper hood right
to left.  Both are pinned here against things other than the oracle itself:
brute-force evaluation of their definitions on small lattices, closed forms,
Qhull on points in general position, and exact invariants.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import brute, invariants


def lower(xy):
    return [int(i) for i in oracle.lower_hull(xy)]


def full(xy):
    return [int(i) for i in oracle.convex_hull(xy)]


def _check_full(xy):
    got = full(xy)
    assert sorted(got) == brute.convex_hull_corners_brute(xy)
    assert invariants.check_convex_hull(xy, got) == []
    return got


# ---------------------------------------------------------------- closed forms
def test_empty_single_and_two_points():
    assert lower(np.zeros((0, 2), np.float32)) == []
    assert full(np.zeros((0, 2), np.float32)) == []
    assert lower([[0.5, 0.25]]) == [0] and full([[0.5, 0.25]]) == [0]
    assert lower([[0.25, 0.5], [0.75, -0.5]]) == [0, 1]
    assert full([[0.25, 0.5], [0.75, -0.5]]) == [0, 1]


def test_vertical_pair_and_duplicates():
    # equal x: the lower hood keeps the lower point, the hull keeps both
    xy = [[0.5, 0.75], [0.5, -0.25]]
    assert lower(xy) == [1]
    assert full(xy) == [1, 0]
    # identical points resolve to the lowest index everywhere
    xy = [[0.5, 0.25], [0.5, 0.25], [0.5, 0.25]]
    assert lower(xy) == [0] and full(xy) == [0]


def test_triangle_and_square_counter_clockwise():
    tri = [[0.0, 0.0], [0.0, 0.5], [1.0, 0.0]]
    assert full(tri) == [0, 2, 1]
    sq = [[0.0, 0.0], [0.0, 1.0], [0.5, 0.5], [1.0, -1.0], [1.0, 1.0]]
    # lowest point of least x, then counter-clockwise; the centre is inside
    assert full(sq) == [0, 3, 4, 1]


def test_collinear_points_keep_the_two_ends():
    xy = synth.from_integers(np.arange(9), 3 * np.arange(9) - 4, 5)
    assert lower(xy) == [0, 8]
    assert full(xy) == [0, 8]


def test_convex_and_concave_sequences():
    K = 40
    X = np.arange(K)
    xy = synth.from_integers(X, X * X, 12)  # strictly convex: every point on the lower hood
    assert lower(xy) == list(range(K))
    assert full(xy) == list(range(K))  # upper hood [0, K-1] adds nothing
    xy = synth.from_integers(X, X * (K - X), 12)  # strictly concave
    assert lower(xy) == [0, K - 1]
    assert full(xy) == [0] + list(range(K - 1, 0, -1))


# ------------------------------------------------------------------ brute force
def _lattice_cases():
    pts = [(x, y) for x in range(3) for y in range(3)]
    seen = set()
    for n in range(1, 6):
        for combo in itertools.product(pts, repeat=n):
            seq = tuple(sorted(combo, key=lambda p: p[0]))
            if seq not in seen:
                seen.add(seq)
                yield seq


def test_brute_force_exhaustive_3x3_up_to_5_points():
    count = 0
    for seq in _lattice_cases():
        xy = synth.from_integers([p[0] for p in seq], [p[1] for p in seq], 2)
        assert lower(xy) == brute.lower_hull_brute(xy), seq
        if len(seq) <= 4:  # the hull's brute force is O(n^4)
            _check_full(xy)
        count += 1
    assert count > 5000


@pytest.mark.parametrize("side", [4, 8, 16])
def test_brute_force_random_lattices(side):
    for seed in range(200):
        n = 1 + seed % 11
        xy = synth.lattice_points(n, side, seed=seed * 37 + side)
        got = lower(xy)
        assert got == brute.lower_hull_brute(xy), (side, seed)
        assert invariants.check_lower(xy, got) == []
        _check_full(xy)


# ---------------------------------------------------------------------- Qhull
@pytest.mark.parametrize("seed", range(6))
def test_qhull_general_position(seed):
    spatial = pytest.importorskip("scipy.spatial")
    rng = np.random.default_rng(100 + seed)
    n = 3000
    X = np.sort(rng.choice(1 << 20, n, replace=False))
    Y = rng.integers(0, 1 << 20, n)
    xy = synth.from_integers(X, Y, 20)
    v = [int(i) for i in spatial.ConvexHull(xy.astype(np.float64)).vertices]  # counter-clockwise
    k = v.index(min(v, key=lambda i: (xy[i, 0], xy[i, 1])))
    assert full(xy) == v[k:] + v[:k]


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("name", ["uniform", "arc", "parabola"])
def test_invariants_on_workload_recipes(name):
    pts = {"uniform": lambda: synth.uniform(1 << 14, 20), "arc": lambda: synth.arc(1 << 14, 24, 4),
           "parabola": lambda: synth.parabola(1 << 12, 20, 1)}[name]()
    assert invariants.check_lower(pts, oracle.lower_hull(pts)) == []
    assert invariants.check_convex_hull(pts, oracle.convex_hull(pts)) == []


def test_invariants_reject_wrong_answers():
    xy = synth.lattice_points(12, 16, seed=5, allow_dup=False)
    good = full(xy)
    assert invariants.check_convex_hull(xy, good) == []
    assert invariants.check_convex_hull(xy, good[::-1]) != []          # clockwise
    assert invariants.check_convex_hull(xy, good[1:] + good[:1]) != []  # wrong start
    assert invariants.check_convex_hull(xy, good[:-1]) != []            # corner missing
    lo = lower(xy)
    assert invariants.check_lower(xy, lo) == []
    assert invariants.check_lower(xy, [int(i) for i in oracle.upper_hull(xy)]) != []


def test_batched_lower_equals_per_set():
    sets = [synth.uniform(500, 20, seed=3), np.zeros((0, 2), np.float32),
            synth.arc(700, 20, 4, seed=4), synth.lattice_points(9, 8, seed=6)]
    pts, off = synth.concat_sets(sets)
    out, cnt = oracle.lower_hull_batched(pts, off)
    for s, xy in enumerate(sets):
        assert list(out[off[s]:off[s] + cnt[s]]) == lower(xy)


def test_error_codes_match_the_upper_hood():
    for bad in ([[0.5, 0.0], [0.25, 0.0]], [[0.5, 2.0 ** -40]], [[1.5, 0.0]]):
        assert oracle.lower_hull_status(bad)[0] == oracle.upper_hull_status(bad)[0] < 0
        assert oracle.convex_hull_status(bad)[0] == oracle.upper_hull_status(bad)[0]
