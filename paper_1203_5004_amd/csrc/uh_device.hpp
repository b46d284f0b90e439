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

// Per-lane counters of orientation tests and exact fallbacks.
struct OrientCount {
  uint32_t evals = 0;
  uint32_t fallbacks = 0;
};

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
__device__ __forceinline__ int orient_sign(float px, float py, float qx,
                                           float qy, float rx, float ry,
                                           OrientCount &cnt, bool force_exact) {
#pragma clang fp contract(off)
  cnt.evals++;
  const float dx1 = qx - px, dy1 = qy - py;
  const float dx2 = rx - px, dy2 = ry - py;
  const float l = dx1 * dy2;
  const float r = dy1 * dx2;
  const float det = l - r;
  const float bound = (__builtin_fabsf(l) + __builtin_fabsf(r)) * 0x1p-22f;
  if (!force_exact && (__builtin_fabsf(det) > bound || bound == 0.0f))
    return (det > 0.0f) - (det < 0.0f);
  cnt.fallbacks++;
  return orient_exact(px, py, qx, qy, rx, ry);
}

__device__ __forceinline__ int orient_sign(float2 p, float2 q, float2 r,
                                           OrientCount &cnt, bool fe) {
  return orient_sign(p.x, p.y, q.x, q.y, r.x, r.y, cnt, fe);
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

// lo + floor(k * span / div) without 32-bit overflow for large spans.
__device__ __forceinline__ int sample_at(int lo, int k, int span, int div) {
  if (span < (1 << 27)) return lo + (k * span) / div;
  return lo + (int)(((long long)k * (long long)span) / div);
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

  int plo = 0, phi = hp;
  for (;;) {
    const int span = phi - plo;
    const int i = sample_at(plo, x, span, d1);
    const float2 p = P[i];
    // mam1/mam2: tangent corner of p on Q, in [lo, hi)
    int lo = 0, hi = hq;
    while (hi - lo > 1) {
      const int sp = hi - lo;
      const int s = sample_at(lo, y + 1, sp, d2 + 1);
      const int gv = g_classify(p, Q, s, hq, cnt, fe);
      const uint32_t ml = (uint32_t)(__ballot(gv == LOW) >> sub) & sub_mask;
      const uint32_t me = (uint32_t)(__ballot(gv == EQUAL) >> sub) & sub_mask;
      const uint32_t mh = (uint32_t)(__ballot(gv == HIGH) >> sub) & sub_mask;
      if (me) {
        lo = sample_at(lo, __builtin_ctz(me) + 1, sp, d2 + 1);
        hi = lo + 1;
        break;
      }
      const int nl = __builtin_popcount(ml);
      const int nh = __builtin_popcount(mh);
      const int nlo = nl ? sample_at(lo, nl, sp, d2 + 1) + 1 : lo;
      const int nhi = nh ? sample_at(lo, d2 - nh + 1, sp, d2 + 1) : hi;
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
      out_a = sample_at(plo, k, span, d1);
      out_b = __shfl(jt, base + k * d2, 64);
      return;
    }
    const int nl = __builtin_popcount(fl);
    const int nh = __builtin_popcount(fh);
    const int nplo = nl ? sample_at(plo, nl - 1, span, d1) + 1 : plo;
    const int nphi = nh ? sample_at(plo, d1 - nh, span, d1) : phi;
    if (nphi <= nplo) {  // only on an inconsistent (invalid-data) predicate
      out_a = nplo < 0 ? 0 : (nplo >= hp ? hp - 1 : nplo);
      out_b = 0;
      return;
    }
    plo = nplo;
    phi = nphi;
  }
}

}  // namespace uh
