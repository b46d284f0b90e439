"""Per-merge quantities of match-and-merge, by brute force -- TEST INFRASTRUCTURE.

The paper merges the hoods H(P) and H(Q) of two adjacent x-ranges by finding
their common tangent ("bridge") and keeping P's corners up to the bridge's
left end and Q's corners from its right end (match-and-merge, steps mam0 to
mam6).  Its classifiers, as described before their code:

  g(p, q): for p left of Q and q a corner of H(Q), LOW / EQUAL / HIGH as q is
           left of / at / right of the corner q' supporting the tangent from
           p to H(Q);
  f(p, q): symmetric -- p a corner of H(P), q right of P, as p is left of /
           at / right of the corner supporting the tangent from q to H(P).

The paper assumes general position, where the supporting corner is unique.
Reading used here for ties (a tangent line through several corners): the
merged chain must stay strictly concave, so the bridge takes the LEFTMOST
P-corner and the RIGHTMOST Q-corner on the common tangent; accordingly the
tangent corner on H(Q) is the rightmost one on the tangent line, and the
tangent corner on H(P) is the leftmost one.

``g_def`` / ``f_def`` / ``bridge`` evaluate these from the definitions (all
corners checked against each candidate line).  ``g_rule`` / ``f_rule`` are the
paper's local neighbour tests (compare the next and previous corners with the
line pq; an end corner's missing neighbour lies directly below it, so it
never triggers) with the tie reading above:

  g: LOW   iff q_next is on or above line p->q,
     HIGH  iff otherwise q_prev is strictly above it, else EQUAL;
  f: LOW   iff p_next is strictly above line p->q,
     HIGH  iff otherwise p_prev is on or above it, else EQUAL.

The tests check that the rules equal the definitions, and the paper's
monotonicity theorem (tangent corners nondecreasing; f at a sample's tangent
corner locates the bridge corner), on exhaustive and random small hoods.

Hoods are lists of exact integer points (X, Y), strictly increasing in X and
strictly concave; every P point lies strictly left of every Q point.
"""
from __future__ import annotations

LOW, EQUAL, HIGH = -1, 0, 1


def det(a, b, c) -> int:
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _sign(v: int) -> int:
    return (v > 0) - (v < 0)


def tangent_corner_on_q(p, Q) -> int:
    """Rightmost j such that every corner of Q is on or below line p -> Q[j]."""
    best = None
    for j in range(len(Q)):
        if all(det(p, Q[j], Q[k]) <= 0 for k in range(len(Q))):
            best = j
    assert best is not None
    return best


def tangent_corner_on_p(q, P) -> int:
    """Leftmost i such that every corner of P is on or below line P[i] -> q."""
    for i in range(len(P)):
        if all(det(P[i], q, P[k]) <= 0 for k in range(len(P))):
            return i
    raise AssertionError("no tangent corner")


def g_def(p, Q, j) -> int:
    return _sign(j - tangent_corner_on_q(p, Q))


def f_def(q, P, i) -> int:
    return _sign(i - tangent_corner_on_p(q, P))


def g_rule(p, Q, j) -> int:
    q = Q[j]
    if j + 1 < len(Q) and det(p, q, Q[j + 1]) >= 0:
        return LOW
    if j > 0 and det(p, q, Q[j - 1]) > 0:
        return HIGH
    return EQUAL


def f_rule(q, P, i) -> int:
    p = P[i]
    if i + 1 < len(P) and det(p, q, P[i + 1]) > 0:
        return LOW
    if i > 0 and det(p, q, P[i - 1]) >= 0:
        return HIGH
    return EQUAL


def bridge(P, Q):
    """(a, b): leftmost P-corner and rightmost Q-corner on the common tangent,
    i.e. on a line through one corner of each with all corners on or below."""
    valid = [(i, j) for i in range(len(P)) for j in range(len(Q))
             if all(det(P[i], Q[j], r) <= 0 for r in list(P) + list(Q))]
    assert valid, "no common tangent"
    return min(i for i, _ in valid), max(j for _, j in valid)


def survivors(P, Q):
    """Corner-wise form of the merge, by definition of a strict corner:
    P corner i stays iff i == 0 or every Q corner is strictly below the line
    through P[i-1] and P[i]; Q corner j stays iff j == last or every P corner
    is strictly below the line through Q[j] and Q[j+1].  Returns the kept
    index sets (they are P[0..a] and Q[b..] for the bridge (a, b))."""
    keep_p = [i for i in range(len(P))
              if i == 0 or all(det(P[i - 1], P[i], q) < 0 for q in Q)]
    keep_q = [j for j in range(len(Q))
              if j == len(Q) - 1 or all(det(Q[j], Q[j + 1], p) < 0 for p in P)]
    return keep_p, keep_q


def merge(P, Q):
    """Corner list of H(P u Q): P[0..a] followed by Q[b..]."""
    a, b = bridge(P, Q)
    return list(P[: a + 1]) + list(Q[b:])
