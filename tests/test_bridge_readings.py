"""Pins for the readings of the paper's match-and-merge step (CPU only).

* the local neighbour tests g / f (with the tie reading: rightmost tangent
  corner on H(Q), leftmost on H(P)) equal their definitions;
* the paper's monotonicity theorem, under that reading, on exhaustive tiny
  hoods and random larger ones, including collinear ties: its second claim
  (f at a sample's tangent corner tells whether the sample is left of, at
  or right of the bridge corner) holds for every sample; its first claim
  (tangent corners nondecreasing) holds for the samples at or left of the
  bridge corner and fails to the right of it, even in general position
  (test_theorem_first_claim_counterexample);
* the merge P[0..a] ++ Q[b..] equals the hood of the union (the oracle);
* the stopping condition of mam5 read as a test on pairs: exactly one pair
  (i, j) has g(P[i], Q[j]) = f(Q[j], P[i]) = EQUAL, and it is the bridge
  defined as the leftmost P-corner and rightmost Q-corner on the common
  tangent (the merge kernels classify all pairs of small hoods this way).
"""
import itertools
import random

import numpy as np
import pytest

import oracle
from oracle import bridge as B


def _hood(points):
    """Strict upper hood of integer points (distinct x), via the oracle."""
    pts = sorted(points)
    xy = np.array(pts, dtype=np.float64) / 64.0
    idx = oracle.upper_hull(xy.astype(np.float32))
    return [pts[i] for i in idx]


def _random_pair(rng, nmax, span=64, collinear_bias=False):
    """Two hoods from random point sets on disjoint x-ranges of a lattice."""
    while True:
        xs = sorted(rng.sample(range(span), rng.randint(2, min(nmax, span))))
        cut = rng.randint(1, len(xs) - 1)
        if collinear_bias:
            slope = rng.randint(-2, 2)
            ys = [min(63, max(0, 20 + slope * x // 4 + rng.choice([0, 0, 0, -1, -3])))
                  for x in xs]
        else:
            ys = [rng.randint(0, 63) for _ in xs]
        P = _hood(list(zip(xs[:cut], ys[:cut])))
        Q = _hood(list(zip(xs[cut:], ys[cut:])))
        return P, Q


def _check_pair(P, Q):
    # local rules equal definitions
    for p in P:
        for j in range(len(Q)):
            assert B.g_rule(p, Q, j) == B.g_def(p, Q, j), (P, Q, p, j)
    for q in Q:
        for i in range(len(P)):
            assert B.f_rule(q, P, i) == B.f_def(q, P, i), (P, Q, q, i)
    # monotonicity theorem
    a, b = B.bridge(P, Q)
    tang = [B.tangent_corner_on_q(p, Q) for p in P]
    assert all(tang[i] <= tang[i + 1] for i in range(a)), (P, Q, tang)
    for i, p in enumerate(P):
        want = (i > a) - (i < a)
        assert B.f_rule(Q[tang[i]], P, i) == want, (P, Q, i, a)
    assert tang[a] == b
    # merge = hood of the union
    assert B.merge(P, Q) == _hood(P + Q)
    # the corner-wise survival test picks exactly P[0..a] and Q[b..]
    kp, kq = B.survivors(P, Q)
    assert kp == list(range(a + 1)) and kq == list(range(b, len(Q))), (P, Q)
    # the pairs classified EQUAL by both g and f: exactly the bridge
    mutual = [(i, j) for i in range(len(P)) for j in range(len(Q))
              if B.g_rule(P[i], Q, j) == B.EQUAL and B.f_rule(Q[j], P, i) == B.EQUAL]
    assert mutual == [(a, b)], (P, Q, mutual)


def test_exhaustive_small_hoods():
    """Every split of every x-sorted set of up to 6 points of a 6x4 lattice
    with distinct x (1 to 3 points per side)."""
    count = 0
    for n in range(2, 7):
        for xs in itertools.combinations(range(6), n):
            for ys in itertools.product(range(4), repeat=n):
                pts = list(zip(xs, ys))
                for cut in range(1, n):
                    P = _hood(pts[:cut])
                    Q = _hood(pts[cut:])
                    if len(P) > 3 or len(Q) > 3:
                        continue
                    _check_pair(P, Q)
                    count += 1
                if count > 6000:
                    return
    assert count > 1000


@pytest.mark.parametrize("collinear", [False, True])
def test_random_hoods(collinear):
    rng = random.Random(5004 + collinear)
    for _ in range(300):
        P, Q = _random_pair(rng, 40, collinear_bias=collinear)
        _check_pair(P, Q)


def test_golden_collinear_bridge_indices():
    P = [(0, 0), (2, 4), (4, 6)]
    Q = [(6, 8), (8, 10), (10, 10)]
    assert B.bridge(P, Q) == (1, 1)
    assert B.merge(P, Q) == [(0, 0), (2, 4), (8, 10), (10, 10)]


def test_theorem_first_claim_counterexample():
    """General position, yet the tangent corners decrease to the right of the
    bridge corner: from (0,100) the tangent touches Q's last corner (slopes
    -10, -8.2, -4.4), from (1,-100) its first (slopes 11.1, 11, 5.9).  The
    classification claim still holds: f says HIGH for the right sample."""
    P = [(0, 100), (1, -100)]
    Q = [(10, 0), (11, 10), (20, 12)]
    tang = [B.tangent_corner_on_q(p, Q) for p in P]
    assert tang == [2, 0]
    assert B.bridge(P, Q) == (0, 2)
    assert B.f_rule(Q[tang[0]], P, 0) == B.EQUAL
    assert B.f_rule(Q[tang[1]], P, 1) == B.HIGH
