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


# -------------------------------------------------------------- unsorted input
def _brute_by_x(xy, corners):
    X, _ = brute.exact_ints(xy)
    return sorted(corners, key=lambda i: X[i])


def test_unsorted_matches_brute_force_on_shuffled_lattices():
    rng = np.random.default_rng(7)
    for seed in range(300):
        xy = synth.lattice_points(1 + seed % 12, (4, 8, 16)[seed % 3], seed=900 + seed)
        sh = xy[rng.permutation(len(xy))]
        rc, up = oracle.unsorted_hull(sh, "upper")
        assert rc == 0 and list(up) == _brute_unsorted(sh)
        # the upper hood's brute force does not depend on the input order either
        assert list(up) == _brute_by_x(sh, brute.upper_hull_brute(sh))
        rc, lo = oracle.unsorted_hull(sh, "lower")
        assert rc == 0 and list(lo) == _brute_unsorted(sh, lower=True)
        if seed % 3 == 0:
            rc, full = oracle.unsorted_hull(sh, "convex")
            assert rc == 0 and sorted(full) == _brute_hull_corners_unsorted(sh)
            assert invariants.check_convex_hull(sh, full) == []


def _brute_unsorted(xy, lower=False):
    """The hood's definition evaluated on points in any order: i is a corner
    iff no point at its x is higher (lower hood: lower), or equally high
    with a lower index, and no pair a, b with X_a < X_i < X_b has i on or
    below (lower hood: on or above) segment ab.  Corners by x."""
    X, Y = brute.exact_ints(xy)
    n = len(X)
    sgn = -1 if lower else 1
    out = []
    for i in range(n):
        if any(j != i and X[j] == X[i] and (sgn * Y[j] > sgn * Y[i] or (Y[j] == Y[i] and j < i))
               for j in range(n)):
            continue
        if any(sgn * brute.det(X, Y, a, b, i) <= 0 for a in range(n) for b in range(n)
               if X[a] < X[i] < X[b]):
            continue
        out.append(i)
    return sorted(out, key=lambda i: X[i])


def _brute_hull_corners_unsorted(xy):
    # the corner set does not depend on the order; ties to the lowest index
    return brute.convex_hull_corners_brute(xy)


def test_unsorted_sorted_input_is_unchanged():
    xy = synth.uniform(5000, 20, seed=8)
    for hood, fn in (("upper", oracle.upper_hull), ("lower", oracle.lower_hull),
                     ("convex", oracle.convex_hull)):
        rc, got = oracle.unsorted_hull(xy, hood)
        assert rc == 0 and np.array_equal(got, fn(xy))


def test_unsorted_tie_rules_follow_input_index():
    # identical points in reverse input order: the lowest input index wins
    xy = np.array([[0.75, 0.5], [0.25, 0.25], [0.75, 0.5], [0.25, 0.25], [0.5, -0.5]], np.float32)
    assert list(oracle.unsorted_hull(xy, "upper")[1]) == [1, 0]
    assert list(oracle.unsorted_hull(xy, "lower")[1]) == [1, 4, 0]
    assert list(oracle.unsorted_hull(xy, "convex")[1]) == [1, 4, 0]
