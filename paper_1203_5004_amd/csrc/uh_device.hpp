// uh_device.hpp -- device building blocks of the upper-hood library (gfx950).
//
//  * orient_sign : the paper's left_of predicate as an exact three-way sign,
//                  FP32 with a forward error-bound filter, exact FP64
//                  re-evaluation when the filter cannot decide;
//  * g_classify / f_classify : the tangent classifiers g and f of
//                  match-and-merge (LOW / EQUAL / HIGH);
//  * bridge_search : the common tangent of two hoods by the paper's sampled
//                  search (P-samples x Q-samples, mam1-mam5), run by the
//                  lanes of one wave64 with ballots.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uh {

enum : int { LOW = -1, EQUAL = 0, HIGH = 1 };

// Per-lane counters of orientation tests and exact fallbacks; with `check`
// every sign is also compared with a 128-bit integer evaluation and
// disagreements are counted (the predicate's soundness check).
struct OrientCount {
  uint32_t evals = 0;
  uint32_t fallbacks = 0;
  uint32_t sign_errors = 0;
  bool check = false;
};

// Sign of det(q - p, r - p) in 128-bit integers: every coordinate on the
// 2^-30 grid is an integer multiple of 2^-30 (scaling by 2^30 and converting
// is exact), so the determinant of the integer coordinates has the exact
// sign.  Used only by the soundness check.
__device__ __noinline__ int orient_int128(float px, float py, float qx, float qy, float rx,
                                          float ry) {
  const long long X0 = (long long)((double)px * 1073741824.0);
  const long long Y0 = (long long)((double)py * 1073741824.0);
  const long long X1 = (long long)((double)qx * 1073741824.0);
  const long long Y1 = (long long)((double)qy * 1073741824.0);
  const long long X2 = (long long)((double)rx * 1073741824.0);
  const long long Y2 = (long long)((double)ry * 1073741824.0);
  const __int128 d = (__int128)(X1 - X0) * (__int128)(Y2 - Y0) -
                     (__int128)(Y1 - Y0) * (__int128)(X2 - X0);
  return (d > 0) - (d < 0);
}

// Exact sign of det(q - p, r - p) for coordinates on the 2^-30 grid with
// x in [0, 1] and y in [-1, 1].
//   - differences are exact in FP64: x-differences are multiples of 2^-30
//     below 1 in magnitude (31 bits), y-differences below 2 (32 bits);
//   - each y-difference is split into a part on the 2^-16 grid (18 bits)
//     and a remainder below 2^-17 (14 bits), so every product of an
//     x-difference with a part needs at most 48 bits: exact;
//   - the two partial determinants are differences of exact products on a
//     common grid, at most 49 and 45 bits wide: exact;
//   - their sum is rounded once, and round-to-nearest keeps the sign (and
//     zero-ness) of an exact value.
__device__ __forceinline__ int orient_exact(float px, float py, float qx,
                                            float qy, float rx, float ry) {
#pragma clang fp contract(off)
  const double dx1 = (double)qx - (double)px;
  const double dy1 = (double)qy - (double)py;
  const double dx2 = (double)rx - (double)px;
  const double dy2 = (double)ry - (double)py;
  const double h1 = __builtin_rint(dy1 * 65536.0) * (1.0 / 65536.0);
  const double h2 = __builtin_rint(dy2 * 65536.0) * (1.0 / 65536.0);
  const double l1 = dy1 - h1;
  const double l2 = dy2 - h2;
  const double hi = dx1 * h2 - h1 * dx2;
  const double lo = dx1 * l2 - l1 * dx2;
  const double det = hi + lo;
  return (det > 0.0) - (det < 0.0);
}

// Sign of det(q - p, r - p): > 0 iff r is left of the directed line p -> q
// (above it when p.x < q.x), as the paper's left_of.
// FP32 filter: with rounding unit u = 2^-24 the computed determinant is
// within (3u + 16u^2)(|l| + |r|) of the exact one (Shewchuk, "Adaptive
// precision floating-point arithmetic and fast robust geometric predicates",
// 1997, orient2d bound A, with binary32's u).  The bound used here,
// (|l| + |r|) * 2^-22, exceeds it even after the rounding of the sum, and
// its multiplication is exact.  No underflow is possible on the grid (the
// smallest non-zero product is 2^-60), so a zero bound means both products
// are exactly zero and so is the determinant.  Contraction into FMA is off:
// the bound assumes separately rounded products.
// A lane that is not `live` (its result will be ignored; for branch-free
// loops) gets the filter's sign, counts nothing and never takes the exact
// path.
__device__ __forceinline__ int orient_sign(float px, float py, float qx,
                                           float qy, float rx, float ry,
                                           OrientCount &cnt, bool force_exact,
                                           bool live = true) {
#pragma clang fp contract(off)
  cnt.evals += live ? 1u : 0u;
  const float dx1 = qx - px, dy1 = qy - py;
  const float dx2 = rx - px, dy2 = ry - py;
  const float l = dx1 * dy2;
  const float r = dy1 * dx2;
  const float det = l - r;
  const float bound = (__builtin_fabsf(l) + __builtin_fabsf(r)) * 0x1p-22f;
  int sg = (det > 0.0f) - (det < 0.0f);
  // bitwise, so that the only branch is the one around the exact path
  const bool decided =
      !live | (!force_exact & ((__builtin_fabsf(det) > bound) | (bound == 0.0f)));
  if (!decided) {
    cnt.fallbacks++;
    sg = orient_exact(px, py, qx, qy, rx, ry);
  }
  if (cnt.check && live && sg != orient_int128(px, py, qx, qy, rx, ry)) cnt.sign_errors++;
  return sg;
}

__device__ __forceinline__ int orient_sign(float2 p, float2 q, float2 r,
                                           OrientCount &cnt, bool fe, bool live = true) {
  return orient_sign(p.x, p.y, q.x, q.y, r.x, r.y, cnt, fe, live);
}

// True only where the FP32 filter of orient_sign certifies that r lies
// strictly right of p -> q (strictly below the line, for p.x < q.x); an
// undecided case gives false.  For tests whose only use of a true answer is
// to drop a point that cannot be a corner, so that undecided points are
// simply kept and no exact evaluation is needed.  With force_exact (the
// ablation that sends every test down the exact path) the exact sign
// decides instead.
__device__ __forceinline__ bool surely_below(float2 p, float2 q, float2 r, OrientCount &cnt,
                                             bool force_exact) {
#pragma clang fp contract(off)
  if (force_exact) return orient_sign(p, q, r, cnt, true) < 0;
  cnt.evals++;
  const float dx1 = q.x - p.x, dy1 = q.y - p.y;
  const float dx2 = r.x - p.x, dy2 = r.y - p.y;
  const float l = dx1 * dy2;
  const float rr = dy1 * dx2;
  const float det = l - rr;
  const float bound = (__builtin_fabsf(l) + __builtin_fabsf(rr)) * 0x1p-22f;
  const bool below = det < -bound;
  if (cnt.check && below && orient_int128(p.x, p.y, q.x, q.y, r.x, r.y) >= 0) cnt.sign_errors++;
  return below;
}

// g(p, q_j): where corner j of the hood Q lies relative to the corner q'
// that supports the tangent from p (p strictly left of Q):
//   LOW   if q_{j+1} is on or above line p -> q_j   (q' is further right),
//   HIGH  else if q_{j-1} is strictly above it      (q' is further left),
//   EQUAL otherwise.
// An end corner's missing neighbour lies directly below it (the paper's
// vertical closure), which never triggers either test.  The on-line case
// counts as LOW, so q' is the RIGHTMOST corner on the tangent line.
template <class PT>
__device__ __forceinline__ int g_classify(float2 p, PT Q, int j, int hq,
                                          OrientCount &cnt, bool fe) {
  const float2 q = Q[j];
  if (j + 1 < hq && orient_sign(p, q, Q[j + 1], cnt, fe) >= 0) return LOW;
  if (j > 0 && orient_sign(p, q, Q[j - 1], cnt, fe) > 0) return HIGH;
  return EQUAL;
}

// f(p_i, q): where corner i of the hood P lies relative to the corner p'
// that supports the tangent from q (q strictly right of P):
//   LOW   if p_{i+1} is strictly above line p_i -> q (p' is further right),
//   HIGH  else if p_{i-1} is on or above it          (p' is further left),
//   EQUAL otherwise.
// The on-line case counts as HIGH, so p' is the LEFTMOST corner on it.
template <class PT>
__device__ __forceinline__ int f_classify(float2 q, PT P, int i, int hp,
                                          OrientCount &cnt, bool fe) {
  const float2 p = P[i];
  if (i + 1 < hp && orient_sign(p, q, P[i + 1], cnt, fe) > 0) return LOW;
  if (i > 0 && orient_sign(p, q, P[i - 1], cnt, fe) >= 0) return HIGH;
  return EQUAL;
}

// Sample positions.  Correctness of the searches below only needs samples
// that are nondecreasing in the lane index and stay inside [lo, lo + span);
// they are computed without integer division (which costs dozens of
// instructions on the GPU):
//   P samples: lo + floor(k * span / d1) with d1 a power of two (a shift);
//   Q samples: lo + floor(span * k * c), c = (1 - 2^-22) / (d2 + 1) < 1 / (d2 + 1),
//              in FP32 while span < 2^24 (exact conversion), else in FP64.
// Every lane evaluates the same expression for the same k, so the bounds
// recomputed from the ballots match the positions the lanes sampled.
__device__ __forceinline__ int psample(int lo, int k, int span, int lg1) {
  if (span < (1 << 26)) return lo + ((k * span) >> lg1);
  return lo + (int)(((long long)k * (long long)span) >> lg1);
}

__device__ __forceinline__ int qsample(int lo, int k, int span, float c, double cd) {
  if (span < (1 << 24)) return lo + (int)((float)span * ((float)k * c));
  return lo + (int)((double)span * ((double)k * cd));
}

// Gather the bits of the d1 sub-group leaders (lanes base + k * d2) of a
// wave ballot into the low d1 bits.
__device__ __forceinline__ uint32_t leader_bits(uint64_t ballot, int base,
                                                int d1, int d2) {
  uint32_t out = 0;
  for (int k = 0; k < d1; ++k)
    out |= (uint32_t)((ballot >> (base + k * d2)) & 1ull) << k;
  return out;
}

// Common tangent (bridge) of two hoods P[0..hp) and Q[0..hq), hp, hq >= 1,
// P strictly left of Q.  Returns a = leftmost P-corner and b = rightmost
// Q-corner on it.
//
// Called together by the L lanes of one group (L a power of two <= 64,
// lanes base .. base + L - 1 of one wave, t = lane - base).  As in the
// paper's thread block, the L lanes form d1 P-samples x d2 lanes per sample
// (d1 = 2^ceil(lg L / 2), d2 = L / d1):
//   mam1/mam2 -- each sample's d2 lanes locate the sample's tangent corner
//     on Q by a (d2+1)-ary search driven by g (one ballot per step);
//   mam3 -- f at each sample's tangent corner classifies the sample as
//     left of / at / right of the bridge corner p (the second claim of the
//     paper's theorem, which holds for every sample); the samples bracket p;
//   mam4/mam5 -- repeated on the bracket until a sample's f is EQUAL: that
//     sample is a and its tangent corner is b.
// Hoods larger than the paper's d1 x d2 block simply take more rounds of
// this bracketing (the multi-level sampling of the paper's conclusions).
// With an exact predicate every step shrinks its interval, so both loops
// end; on invalid data (NaN) they still end and indices stay in range.
template <class PT>
__device__ __forceinline__ void bridge_search(PT P, int hp, PT Q, int hq,
                                              int L, int t, int base,
                                              int &out_a, int &out_b,
                                              OrientCount &cnt, bool fe) {
  const int lg = 31 - __builtin_clz((unsigned)L);
  const int lg1 = (lg + 1) >> 1;
  const int d1 = 1 << lg1;
  const int d2 = L >> lg1;
  const int x = t >> (lg - lg1);
  const int y = t & (d2 - 1);
  const int sub = base + x * d2;
  const uint32_t sub_mask = (1u << d2) - 1u;
  const float c = (1.0f - 0x1p-22f) / (float)(d2 + 1);
  const double cd = (1.0 - 0x1p-40) / (double)(d2 + 1);

  int plo = 0, phi = hp;
  for (;;) {
    const int span = phi - plo;
    const int i = psample(plo, x, span, lg1);
    const float2 p = P[i];
    // mam1/mam2: tangent corner of p on Q, in [lo, hi)
    int lo = 0, hi = hq;
    while (hi - lo > 1) {
      const int sp = hi - lo;
      const int s = qsample(lo, y + 1, sp, c, cd);
      const int gv = g_classify(p, Q, s, hq, cnt, fe);
      const uint32_t ml = (uint32_t)(__ballot(gv == LOW) >> sub) & sub_mask;
      const uint32_t me = (uint32_t)(__ballot(gv == EQUAL) >> sub) & sub_mask;
      const uint32_t mh = (uint32_t)(__ballot(gv == HIGH) >> sub) & sub_mask;
      if (me) {
        lo = qsample(lo, __builtin_ctz(me) + 1, sp, c, cd);
        hi = lo + 1;
        break;
      }
      const int nl = __builtin_popcount(ml);
      const int nh = __builtin_popcount(mh);
      const int nlo = nl ? qsample(lo, nl, sp, c, cd) + 1 : lo;
      const int nhi = nh ? qsample(lo, d2 - nh + 1, sp, c, cd) : hi;
      lo = nlo;
      hi = nhi;
    }
    const int jt = lo < 0 ? 0 : (lo >= hq ? hq - 1 : lo);
    // mam3: classify the samples against the bridge corner
    const int fv = f_classify(Q[jt], P, i, hp, cnt, fe);
    const uint64_t bl = __ballot(fv == LOW);
    const uint64_t be = __ballot(fv == EQUAL);
    const uint64_t bh = __ballot(fv == HIGH);
    const uint32_t fl = leader_bits(bl, base, d1, d2);
    const uint32_t feq = leader_bits(be, base, d1, d2);
    const uint32_t fh = leader_bits(bh, base, d1, d2);
    if (feq) {
      const int k = __builtin_ctz(feq);
      out_a = psample(plo, k, span, lg1);
      out_b = __shfl(jt, base + k * d2, 64);
      return;
    }
    const int nl = __builtin_popcount(fl);
    const int nh = __builtin_popcount(fh);
    const int nplo = nl ? psample(plo, nl - 1, span, lg1) + 1 : plo;
    const int nphi = nh ? psample(plo, d1 - nh, span, lg1) : phi;
    if (nphi <= nplo) {  // only on an inconsistent (invalid-data) predicate
      out_a = nplo < 0 ? 0 : (nplo >= hp ? hp - 1 : nplo);
      out_b = 0;
      return;
    }
    plo = nplo;
    phi = nphi;
  }
}

// The bridge test of mam5 on one pair: true iff P[i] and Q[j] are each
// other's tangent corner, g(P[i], Q[j]) = f(Q[j], P[i]) = EQUAL (with the tie
// rules of g_classify / f_classify the pair is unique).  A missing neighbour
// takes no test: it would compare a corner with itself, an exact zero that
// the filter cannot certify.
template <class PT>
__device__ __forceinline__ bool bridge_pair(PT P, int hp, PT Q, int hq, int i, int j,
                                            OrientCount &oc, bool fe) {
  const int im = i > 0 ? i - 1 : 0, ip = i + 1 < hp ? i + 1 : i;
  const int jm = j > 0 ? j - 1 : 0, jp = j + 1 < hq ? j + 1 : j;
  const float2 pi = P[i], pp = P[im], pn = P[ip];
  const float2 qj = Q[j], qp = Q[jm], qn = Q[jp];
  const bool g_eq = !(j + 1 < hq && orient_sign(pi, qj, qn, oc, fe) >= 0) &&
                    !(j > 0 && orient_sign(pi, qj, qp, oc, fe) > 0);
  return g_eq && !(i + 1 < hp && orient_sign(pi, qj, pn, oc, fe) > 0) &&
         !(i > 0 && orient_sign(pi, qj, pp, oc, fe) >= 0);
}

// The bridge of two hoods (as bridge_search, same lanes), looked for first
// next to the junction, where it nearly always lies once the hoods are
// large and smooth (the late rounds of hull-heavy data); only if it is not
// found there does the sampled search run.
//  - With 8 lanes or more: first P's last wp corners against Q's first wq,
//    one pair per lane (wp * wq = L), each pair given mam5's test
//    (bridge_pair).  If none passes, tangent steps that alternate between
//    the hoods: the L lanes classify Q's corners b .. b + L - 1 with g
//    against P[a] and take the EQUAL one as the new b (the tangent corner of
//    P[a], which lies at or right of b), then P's corners a .. a - L + 1
//    with f against Q[b] for the new a, and so on from the junction pair
//    (hp - 1, 0).  A step after the first that leaves its corner where it
//    was ends the walk: then g(P[a], Q[b]) and f(Q[b], P[a]) are both
//    EQUAL, mam5's test, which only the bridge passes.  A step that finds
//    no EQUAL corner in its window, or PINGPONG_MAX steps without an end,
//    leave it to the search.  (The window costs one step and catches the
//    bridges within sqrt(L) corners of the junction; the tangent steps
//    cover L corners on either side in two or three.)
//  - With fewer: the group's first lane walks from the junction, at most
//    WALK_MAX steps: Q's corner moves right while the next one is on or
//    above the line P[a] -> Q[b] (g is LOW), P's moves left while the
//    previous one is on or above it (f is HIGH).  On x-separated upper
//    hoods such moves never make g HIGH or f LOW, so a walk that stops
//    ends on the bridge; the end pair is checked with bridge_pair all the
//    same, and a walk cut off by the step limit is not used.
constexpr int WALK_MAX = 16;
constexpr int PINGPONG_MAX = 8;

template <class PT>
__device__ __forceinline__ void bridge_find(PT P, int hp, PT Q, int hq, int L, int t, int base,
                                            int &out_a, int &out_b, OrientCount &cnt, bool fe) {
  if (L < 8) {
    int wa = hp - 1, wb = 0, ok = 0;
    if (t == 0) {
      int steps = 0;
      bool moved = true;
      while (moved && steps < WALK_MAX) {
        moved = false;
        while (wb + 1 < hq && steps < WALK_MAX &&
               orient_sign(P[wa], Q[wb], Q[wb + 1], cnt, fe) >= 0) {
          ++wb;
          ++steps;
          moved = true;
        }
        while (wa > 0 && steps < WALK_MAX && orient_sign(P[wa], Q[wb], P[wa - 1], cnt, fe) >= 0) {
          --wa;
          ++steps;
          moved = true;
        }
      }
      ok = bridge_pair(P, hp, Q, hq, wa, wb, cnt, fe) ? 1 : 0;
    }
    ok = __shfl(ok, base, 64);
    if (ok) {
      out_a = __shfl(wa, base, 64);
      out_b = __shfl(wb, base, 64);
      return;
    }
  } else {
    const uint64_t gm = L == 64 ? ~0ull : ((1ull << L) - 1ull);
    {  // the window: one pair per lane
      const int lg = 31 - __builtin_clz((unsigned)L);
      const int lgq = lg >> 1;  // wq = 2^floor(lg / 2), wp = L / wq
      const int i = hp - 1 - (t >> lgq), j = t & ((1 << lgq) - 1);
      const bool hit = i >= 0 && j < hq && bridge_pair(P, hp, Q, hq, i, j, cnt, fe);
      const uint64_t m = (__ballot(hit) >> base) & gm;
      if (m) {
        const int k = __builtin_ctzll(m);
        out_a = hp - 1 - (k >> lgq);
        out_b = k & ((1 << lgq) - 1);
        return;
      }
    }
    int wa = hp - 1, wb = 0;  // tangent steps from the junction
    for (int step = 0; step < PINGPONG_MAX; ++step) {
      bool eq = false;
      if ((step & 1) == 0) {  // Q's side: the tangent corner of P[wa]
        const int j = wb + t;
        eq = j < hq && g_classify(P[wa], Q, j, hq, cnt, fe) == EQUAL;
      } else {                // P's side: the tangent corner of Q[wb]
        const int i = wa - t;
        eq = i >= 0 && f_classify(Q[wb], P, i, hp, cnt, fe) == EQUAL;
      }
      const uint64_t m = (__ballot(eq) >> base) & gm;
      if (!m) break;  // not within L corners: the search decides
      const int k = __builtin_ctzll(m);
      if (k == 0 && step > 0) {  // no move: both classifiers EQUAL here
        out_a = wa;
        out_b = wb;
        return;
      }
      if ((step & 1) == 0) wb += k;
      else wa -= k;
    }
  }
  bridge_search<PT>(P, hp, Q, hq, L, t, base, out_a, out_b, cnt, fe);
}

// Orders LDS accesses of one wave: all lanes' earlier accesses are done
// before any later one (a wave runs in lockstep; this stops the compiler
// from moving LDS operations across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Moves n (x, y, id) records from src to dst inside one LDS region, with the
// G lanes of one group (t = lane in group), correct for overlapping ranges:
// each chunk is read by all lanes before any lane writes it, and chunks go
// left to right for a move to the left, right to left for a move right.
template <class ID>
__device__ __forceinline__ void group_move(float2 *xy, ID *id, int src, int dst,
                                           int n, int lgG, int t) {
  if (n <= 0 || src == dst) return;
  const int G = 1 << lgG;
  const int nch = (n + G - 1) >> lgG;
  for (int k = 0; k < nch; ++k) {
    const int c = dst < src ? k : nch - 1 - k;
    const int e = (c << lgG) + t;
    const bool mine = e < n;
    float2 v = make_float2(0.f, 0.f);
    ID vi = 0;
    if (mine) {
      v = xy[src + e];
      vi = id[src + e];
    }
    wave_sync();
    if (mine) {
      xy[dst + e] = v;
      id[dst + e] = vi;
    }
    wave_sync();
  }
}

// Merge (match-and-merge, mam1-mam6) of two adjacent hoods stored in one LDS
// region: P = [bp, bp + hp) and Q = [bq, bq + hq), bp + hp <= bq, run by the
// G <= 64 lanes of one group of one wave.  The merged hood
// P[0..a] ++ Q[b..] is made contiguous by moving the shorter of the two kept
// parts next to the other; returns its start nb and length nc.
// Also applies the vertical-closure rule at the junction: if P's last and
// Q's first corner share x, only the higher survives (ties: P's, the lower
// index).
//
// The bridge (a, b) is the one pair of corners that are each other's tangent
// corner: g(P[a], Q[b]) and f(Q[b], P[a]) are both EQUAL (the stopping
// condition of mam5; with the tie rules of g and f the pair is unique).
// When hp * hq is at most 4 G, every pair is classified directly, G pairs at
// a time, one pair per lane; larger hoods use the sampled search.
template <class ID>
__device__ __forceinline__ void merge_blocks(float2 *xy, ID *id, int bp, int hp,
                                             int bq, int hq, int lgG, int t, int gbase,
                                             int &nb, int &nc, OrientCount &oc,
                                             bool fe) {
  const int G = 1 << lgG;
  nb = bp;
  nc = hp;
  if (hq == 0) return;
  if (hp > 0) {
    const float2 pl = xy[bp + hp - 1], qf = xy[bq];
    if (pl.x == qf.x) {
      if (qf.y > pl.y)
        --hp;
      else {
        ++bq;
        --hq;
      }
    }
  }
  if (hp == 0) {
    nb = bq;
    nc = hq;
    return;
  }
  if (hq == 0) {
    nc = hp;
    return;
  }
  int a = hp - 1, b = 0;
  const int npair = hp * hq;
  if (npair <= 4 * G) {
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    // pair r = i * hq + j; i = floor((r + 1/2) / hq) in FP32 is exact here
    // (r < 256: the quotient stays at least 1/(2 hq) away from an integer)
    const float rq = 1.0f / (float)hq;
    for (int r0 = 0; r0 < npair; r0 += G) {
      const int r = r0 + t;
      bool hit = false;
      int i = 0, j = 0;
      if (r < npair) {
        i = (int)(((float)r + 0.5f) * rq);
        j = r - i * hq;
        hit = bridge_pair<const float2 *>(xy + bp, hp, xy + bq, hq, i, j, oc, fe);
      }
      const uint64_t m = (__ballot(hit) >> gbase) & gmask;
      if (m) {
        const int k = r0 + __builtin_ctzll(m);
        a = (int)(((float)k + 0.5f) * rq);
        b = k - a * hq;
        break;
      }
    }
  } else {
    bridge_find<const float2 *>(xy + bp, hp, xy + bq, hq, G, t, gbase, a, b, oc, fe);
  }
  const int np = a + 1, nq = hq - b;
  nc = np + nq;
  if (np <= nq) {  // P's kept corners move right, to end just before Q[b]
    nb = bq + b - np;
    group_move(xy, id, bp, nb, np, lgG, t);
  } else {         // Q's kept corners move left, to follow P[a]
    nb = bp;
    group_move(xy, id, bq + b, bp + np, nq, lgG, t);
  }
}

// Serial monotone chain (upper half) over n points stored at xy / id in
// x order, in place: afterwards the first `return value` entries are the
// strict upper hood of the n points (the paper's serial strip hood).  Equal
// x: only the highest point can stay, ties keep the earlier (lower index)
// one.  Works on LDS or global memory (one thread owns the range).
template <class PT, class IT>
__device__ __forceinline__ int chain_inplace(PT xy, IT id, int n, OrientCount &oc, bool fe) {
  int cnt = 0;
  float2 t1 = make_float2(0.f, 0.f), t2 = t1;  // stack top, second
  // points are read eight at a time ahead of the stack's writes, which only
  // ever go to positions at or below the point being read
  for (int i0 = 0; i0 < n; i0 += 8) {
    float2 w8[8];
    decltype(id[0] + 0) i8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (i0 + u < n) {
        w8[u] = xy[i0 + u];
        i8[u] = id[i0 + u];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (i0 + u >= n) break;
      const float2 r = w8[u];
      if (cnt >= 1 && r.x == t1.x) {
        if (r.y <= t1.y) continue;  // the top hides r
        --cnt;                      // r hides the top
        t1 = t2;
        if (cnt >= 2) t2 = xy[cnt - 2];
      }
      while (cnt >= 2 && orient_sign(t2, t1, r, oc, fe) >= 0) {
        --cnt;  // the top is on or below t2 -> r
        t1 = t2;
        if (cnt >= 2) t2 = xy[cnt - 2];
      }
      xy[cnt] = r;
      id[cnt] = i8[u];
      t2 = t1;
      t1 = r;
      ++cnt;
    }
  }
  return cnt;
}

// Rounds of Wagener merges over nleaf <= 64 leaf hoods, run by one whole
// wave: lane l holds leaf l's (base, count) in `blk` (l < nleaf), the leaves
// being consecutive, x-adjacent, non-empty hoods in the LDS arrays xy / id.
// Round j joins blocks of 2^j leaves; with M merges in a round each merge
// gets 64 / M lanes (the paper's d1 x d2 block).  The leaf table stays in
// registers: a merge reads its two blocks from their lanes and its result
// goes back to the lane of its first block.  Returns the hood of all leaves
// (base, count) in every lane.
template <class ID>
__device__ __forceinline__ int2 wave_rounds(float2 *xy, ID *id, int2 blk, int nleaf,
                                            OrientCount &oc, bool fe) {
  const int lane = threadIdx.x & 63;
  int lgn = 0;
  while ((1 << lgn) < nleaf) ++lgn;
#pragma unroll 1
  for (int j = 0; j < lgn; ++j) {
    const int lgG = 6 - lgn + j + 1;
    const int t = lane & ((1 << lgG) - 1);
    const int lp = (lane >> lgG) << (j + 1);  // < 2^lgn <= 64
    const int lq = lp + (1 << j);
    const int2 P = make_int2(__shfl(blk.x, lp, 64), __shfl(blk.y, lp, 64));
    const int2 Q = make_int2(__shfl(blk.x, lq & 63, 64), __shfl(blk.y, lq & 63, 64));
    int nb = P.x, nc = P.y;
    if (lq < nleaf) merge_blocks(xy, id, P.x, P.y, Q.x, Q.y, lgG, t, lane - t, nb, nc, oc, fe);
    wave_sync();
    // lane l, the first block of merge l >> (j + 1), takes that merge's
    // result from the merge's first lane (unchanged where it had no partner)
    const int src = ((lane >> (j + 1)) << lgG) & 63;
    const int rb = __shfl(nb, src, 64), rc = __shfl(nc, src, 64);
    if ((lane & ((2 << j) - 1)) == 0) blk = make_int2(rb, rc);
  }
  return make_int2(__shfl(blk.x, 0, 64), __shfl(blk.y, 0, 64));
}

}  // namespace uh
