"""The bridge finder's alternating tangent steps stop only on the bridge (CPU).

With L lanes, the finder starts from the junction pair (a, b) = (hp - 1, 0)
of two x-separated upper hoods P and Q and alternates
  - a Q step: classify Q[b], ..., Q[b + L - 1] with g against P[a]; the
    lowest EQUAL one becomes b;
  - a P step: classify P[a], ..., P[a - L + 1] with f against Q[b]; the
    lowest-offset EQUAL one becomes a;
a step after the first that leaves its corner in place ends the search with
(a, b); a step with no EQUAL corner in its window, or 8 steps without an
end, hand the merge to the sampled search.
Claims checked here, against the bridge read off a brute-force hood of the
union (the last kept corner of P, the first kept corner of Q; on the
recipe slices the hoods come from the oracle's monotone chain, which is
pinned against the brute force elsewhere):
  - every pair the steps end on is the bridge (the end condition is mam5's
    test, g and f both EQUAL, which only the bridge passes);
  - on hoods of smooth hull-heavy data (slices of the arc and parabola
    recipes), whose bridges lie a few corners from the junction, the steps
    end on the bridge for every merge at L = 16 and L = 64.
g and f are restated from their definitions with exact integer signs and
the tie rules of the kernels: g counts the on-line case as LOW (the tangent
corner is the rightmost on the line), f as HIGH (the leftmost).

This is a specification test of the rule itself; it does not execute the
kernel.
"""
import numpy as np
import pytest

import oracle
import oracle.brute as brute
import synth

LOW, EQUAL, HIGH = -1, 0, 1


def _sign(X, Y, p, q, r):
    d = (X[q] - X[p]) * (Y[r] - Y[p]) - (Y[q] - Y[p]) * (X[r] - X[p])
    return (d > 0) - (d < 0)


def g_class(X, Y, p, Q, j):
    """Where Q[j] lies relative to the tangent corner of p on Q."""
    if j + 1 < len(Q) and _sign(X, Y, p, Q[j], Q[j + 1]) >= 0:
        return LOW
    if j > 0 and _sign(X, Y, p, Q[j], Q[j - 1]) > 0:
        return HIGH
    return EQUAL


def f_class(X, Y, q, P, i):
    """Where P[i] lies relative to the tangent corner of q on P."""
    if i + 1 < len(P) and _sign(X, Y, P[i], q, P[i + 1]) > 0:
        return LOW
    if i > 0 and _sign(X, Y, P[i], q, P[i - 1]) >= 0:
        return HIGH
    return EQUAL


def pingpong(X, Y, P, Q, L, max_steps=8):
    a, b = len(P) - 1, 0
    for step in range(max_steps):
        if step % 2 == 0:
            hits = [t for t in range(L) if b + t < len(Q) and g_class(X, Y, P[a], Q, b + t) == EQUAL]
        else:
            hits = [t for t in range(L) if a - t >= 0 and f_class(X, Y, Q[b], P, a - t) == EQUAL]
        if not hits:
            return None
        k = hits[0]
        if k == 0 and step > 0:
            return a, b
        if step % 2 == 0:
            b += k
        else:
            a -= k
    return None


def brute_bridge(xy, P, Q, hood=brute.upper_hull_brute):
    H = set(int(v) for v in hood(xy))
    a = max(i for i, v in enumerate(P) if v in H)
    b = min(j for j, v in enumerate(Q) if v in H)
    return a, b


def _split_hoods(xy, cut, hood=brute.upper_hull_brute):
    """Hoods of the points left of x = cut and at or right of it (indices into xy)."""
    X, _ = brute.exact_ints(xy)
    left = [i for i in range(len(xy)) if X[i] < cut]
    right = [i for i in range(len(xy)) if X[i] >= cut]
    if not left or not right:
        return None
    P = [left[int(k)] for k in hood(xy[left])]
    Q = [right[int(k)] for k in hood(xy[right])]
    return P, Q


@pytest.mark.parametrize("seed", range(200))
@pytest.mark.parametrize("L", [8, 16, 64])
def test_pingpong_ends_only_on_the_bridge(seed, L):
    rng = np.random.default_rng(seed)
    side = int(rng.choice([4, 8, 16, 32]))
    xy = synth.lattice_points(int(rng.integers(4, 60)), side, seed=seed)
    X, Y = brute.exact_ints(xy)
    xs = sorted(set(X))
    if len(xs) < 2:
        return
    cut = xs[int(rng.integers(1, len(xs)))]
    hoods = _split_hoods(xy, cut)
    if hoods is None:
        return
    P, Q = hoods
    got = pingpong(X, Y, P, Q, L)
    if got is not None:
        assert got == brute_bridge(xy, P, Q)


@pytest.mark.parametrize("L", [16, 64])
@pytest.mark.parametrize("make", [
    lambda s: synth.arc(4096, 24, 4, seed=s),
    lambda s: synth.parabola(4096, 20, 1, seed=s),
])
def test_pingpong_finds_smooth_bridges(make, L):
    for s in range(3):
        xy = make(s)
        X, Y = brute.exact_ints(xy)
        Xs = sorted(X)
        for q in range(1, 8):  # merges at several places along the curve
            cut = Xs[q * len(Xs) // 8]
            P, Q = _split_hoods(xy, cut, oracle.upper_hull)
            got = pingpong(X, Y, P, Q, L)
            assert got == brute_bridge(xy, P, Q, oracle.upper_hull)
