"""The merge kernel's direct corner test equals the hood's definition (CPU).

A merge that keeps at most 64 corners in all is finished by one wave: lane c
takes entry c and keeps it iff
  (i)  no entry at its x is higher, or as high with a lower index, and
  (ii) there is no entry strictly left of it, or none strictly right of it,
       or it lies strictly above the segment from its left tangent point to
       its right tangent point -- the left tangent point found by a scan
       over the entries strictly left of it that replaces the current one
       by q whenever q lies strictly left of the directed line current -> c,
       the right one by a scan over the entries strictly right of it that
       replaces the current one by q whenever q lies strictly left of the
       directed line c -> current.
Claim: the kept entries are exactly the corners of the strict upper hood of
all entries (same indices, lowest index among identical points), i.e. the
brute-force definition.  Checked here on small lattices with many ties,
duplicates, equal-x runs and collinear runs, with the scans in the kernel's
order (entries in index order).

This is a specification test of the rule itself; it does not execute the
kernel.
"""
import numpy as np
import pytest

import oracle.brute as brute
import synth


def direct_corners(xy):
    X, Y = brute.exact_ints(xy)
    n = len(X)

    def orient(a, b, c):  # sign of det(b - a, c - a) on exact integers
        d = (X[b] - X[a]) * (Y[c] - Y[a]) - (Y[b] - Y[a]) * (X[c] - X[a])
        return (d > 0) - (d < 0)

    kept = []
    for c in range(n):
        hidden, lt, rt = False, None, None
        for q in range(n):
            if X[q] == X[c]:
                hidden = hidden or Y[q] > Y[c] or (Y[q] == Y[c] and q < c)
            elif X[q] < X[c]:
                if lt is None or orient(lt, c, q) > 0:
                    lt = q
            else:
                if rt is None or orient(c, rt, q) > 0:
                    rt = q
        if not hidden and (lt is None or rt is None or orient(lt, rt, c) > 0):
            kept.append(c)
    return kept


@pytest.mark.parametrize("seed", range(300))
def test_direct_test_equals_definition_small(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 48))
    side = int(rng.choice([2, 4, 8, 16, 32]))
    xy = synth.lattice_points(n, side, seed=seed)  # ties, duplicates, collinear runs
    assert direct_corners(xy) == brute.upper_hull_brute(xy)


@pytest.mark.parametrize("seed", range(20))
def test_direct_test_on_recipe_slices(seed):
    for make in (lambda: synth.uniform(64, 20, seed=seed),
                 lambda: synth.parabola(64, 20, 1, seed=seed),
                 lambda: synth.uniform_iid(64, 27, seed=seed)):
        xy = make()
        assert direct_corners(xy) == brute.upper_hull_brute(xy)
