"""The tile kernel's exact elimination test never removes a corner (CPU).

Rule (applied per tile before the strip hoods): a point r may be dropped
when some earlier point has y >= r.y and some later point has y > r.y.  The
kernel uses two forms of the witnesses: prefix/suffix maxima over strips of
a tile (any earlier/later point qualifies).  Claim: the hood of the kept
points, with the same tie rules, has exactly the corners of the hood of all
points -- same indices, including the lowest-index rule for identical
points.  Checked here with the oracle on adversarial small inputs (ties,
duplicates, equal-x runs, collinear runs) and on the workload recipes.

This is a specification test of the rule itself; it does not execute the
kernel.
"""
import numpy as np
import pytest

import oracle
import synth


def kept_mask(xy, strip=4):
    """Kept points under the rule, with witnesses restricted to strips of
    `strip` points for the 'later' side (as in the kernel: later strips'
    maxima only) and full prefix for the 'earlier' side."""
    y = np.asarray(xy, np.float32)[:, 1].astype(np.float64)
    n = len(y)
    keep = np.zeros(n, bool)
    nst = (n + strip - 1) // strip
    smax = np.full(nst, -np.inf)
    for s in range(nst):
        smax[s] = y[s * strip:(s + 1) * strip].max()
    for i in range(n):
        s = i // strip
        before = y[:i].max() if i > 0 else -np.inf
        later = smax[s + 1:].max() if s + 1 < nst else -np.inf
        keep[i] = y[i] > before or y[i] >= later
    return keep


def hull_of_kept(xy, keep):
    idx = np.nonzero(keep)[0]
    sub = oracle.upper_hull(xy[idx])
    return idx[sub]


@pytest.mark.parametrize("seed", range(400))
def test_rule_preserves_corners_small(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    side = int(rng.choice([2, 4, 8]))
    xy = synth.lattice_points(n, side, seed=seed)  # many ties and duplicates
    strip = int(rng.choice([1, 2, 3, 4, 16]))
    keep = kept_mask(xy, strip)
    assert list(hull_of_kept(xy, keep)) == list(oracle.upper_hull(xy))


def test_rule_on_recipes():
    for xy in (synth.uniform(20000, 20, seed=1), synth.uniform_iid(20000, 27, seed=2),
               synth.arc(20000, 20, 4, seed=3), synth.parabola(20000, 20, 1, seed=4)):
        keep = kept_mask(xy, 16)
        assert list(hull_of_kept(xy, keep)) == list(oracle.upper_hull(xy))


def test_rule_drops_most_uniform_points():
    xy = synth.uniform(4096, 20, seed=5)
    assert kept_mask(xy, 16).sum() < 60
