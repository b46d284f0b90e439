// wagener_hull.hip -- kernels, schedule and C ABI of the upper-hood library.
//
// Paper: C. O Dunlaing, "CUDA implementation of Wagener's 2D convex hull PRAM
// algorithm".  The paper's program copies the padded hood array to the GPU,
// launches match_and_merge once per stage (d = 2, 4, ..., n/2) and copies it
// back after every stage.  Here the same rounds of pairwise hood merges run
// device-resident, in three kinds of launch enqueued back to back:
//
//   init_kernel   clears the stats counters and writes the counts of empty
//                 sets (launched only when a run needs either).
//   tile_kernel   one wave per tile of T = 64 * K points of one set:
//                 coalesced load with the contract checks, strips of K
//                 consecutive points per lane, an exact elimination of
//                 points that cannot be corners; few survivors leave as a
//                 sorted point list, otherwise each lane builds the hood of
//                 its strip serially (the first step of the paper's
//                 work-optimal variant in its conclusions) and up to six
//                 rounds of Wagener merges of adjacent strip hoods run in
//                 LDS, each merge finding its bridge with the lanes of the
//                 wave and compacting P[0..a] ++ Q[b..]; the tile's result
//                 goes to the workspace (or straight to the output for a
//                 one-tile set).
//   merge_kernel  one workgroup merges up to F consecutive hoods of the
//                 previous level of one set through log2(F) further rounds,
//                 in LDS when they fit, else over the workspace by
//                 narrowing each child's kept interval.  Repeated until
//                 every set has a single hood.
//
// With both hoods the tile kernel also builds, from the same registers, the
// lower hood (the upper hood of the mirrored points) into a second half of
// the schedule; points in any order first go through the device sort in
// radix_sort.hip, and unsort_kernel maps the corners back to input indices.
//
// Hoods are stored compactly (no REMOTE padding): a block's corners are a
// prefix of its slot, with a count.  The workspace holds, at each point's
// position, at most one corner (x, y) and its set-relative index, so one
// block's hood never leaves the slot of the points it covers.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "radix_sort.hpp"
#include "uh_device.hpp"
#include "wagener_hull.h"

namespace uh {

constexpr int BLOCK = 256;       // threads per merge workgroup (4 waves)
constexpr int WIDE = 512;        // threads of the last merge of a set with 257 .. 512 children
constexpr int VMAX = 6144;       // corners a merge workgroup keeps in LDS (two per CU)
constexpr int VMAX_WIDE = 12000; // ... and the wide one (one per CU)
// Bit 31 of a tile's output count: the tile wrote its surviving points (a
// sorted point list, not yet a hood); the merge kernel makes it a hood.
constexpr uint32_t POINTS_FLAG = 0x80000000u;
constexpr int TILE_LIST_MAX = 64;  // most survivors a tile hands on as a list
constexpr int DIRECT_MAX = 64;     // corners a merge finishes by the direct corner test
// A group's maximum owns a 256-byte line of its own, so the atomics of the
// tiles of different groups never queue behind one another.  (The second
// word of a set's first group is the counter of a replicated last merge.)
constexpr int GROUP_STRIDE = 64;

struct TileItem {    // one tile of the tile pass (everything a tile needs: 32 bytes)
  int64_t start;     // first point (absolute)
  int32_t len;       // points, 1 .. T
  int32_t set;
  int32_t rel0;      // start minus the set's start (set-relative index of the first point)
  int16_t nb_lo;     // points of the set just before the tile used as witnesses, 0 .. 16
  int16_t nb_hi;     // points of the set just after it used as witnesses, 0 .. 16
  int32_t set_len;   // points in the tile's set (the tile is the set's only one iff
                     // rel0 == 0 and len == set_len)
  int32_t group;     // the first-level merge item that takes this tile (-1: none)
};

struct MergeItem {   // one workgroup of a merge pass
  int64_t off;       // slot start = first child's slot start (absolute)
  int64_t stride;    // child k's slot starts at off + k * stride
  int32_t child0;    // first child in the previous level's arrays
  int32_t nch;       // children, 1 .. F
  int32_t set;
  int32_t final_;    // 1 if this is its set's last merge
  int32_t g0, ng;    // the set's first-level merge items ("groups"): first, count
  int32_t level;     // 0: the children are tiles, 1: groups, 2: deeper
  int32_t pad;
};

// A merge pass of a single-set run (both hoods: two mirrored sets of the
// same size): its items follow from their index, so no table is read.
struct PassArgs {
  int64_t stride;    // child k of an item starts at off + k * stride
  int32_t children;  // blocks of the previous level per set
  int32_t fan;       // children per item (the last item takes the rest)
  int32_t items;     // items per set in this pass
  int32_t level;     // as MergeItem::level
  int32_t groups;    // first-level items per set
  int32_t pad;
};

struct RunArgs {
  const float2 *pts;
  const int64_t *set_start;  // [S + 1]
  float2 *ws_xy;             // [N] corner coordinates at their slots
  int32_t *ws_idx;           // [N] set-relative index of each corner
  int32_t *set_status;       // [S] worst data error seen (0 = none)
  int32_t *out_idx;
  int32_t *out_counts;
  upper_hull_stats *stats;   // [S] or null
  int64_t n_total;           // points over all sets (workspace length)
  int32_t tile_len;          // T
  int32_t one_set;           // 1: a single set, whose tiles follow from the tile index
  int32_t group_fan;         //    ... and tile t belongs to group t / group_fan
  uint32_t *tile_max;        // [tiles] each tile's highest y (order-preserving code)
  uint32_t *group_max;       // [groups * GROUP_STRIDE] the highest y over each group's tiles (0: none)
  uint32_t flags;
  int64_t n_points;          // input points (n_total, or half of it with both hoods)
  // Both hoods: the lower hood of input set s is set s + lower_sets, its
  // slots are the upper hood's plus lower_n, its tiles and groups are the
  // upper ones' plus lower_tiles / lower_groups (all 0 otherwise).
  int64_t lower_n;
  int32_t lower_tiles, lower_groups, lower_sets;
};

// ------------------------------------------------------------ small helpers
__device__ __forceinline__ int check_point(float2 v) {
  // data contract: x in [0,1], y in [-1,1] (NaN fails both), both on the
  // 2^-30 grid: scaling by 2^30 is exact, and then no fraction may remain
  if (!(v.x >= 0.0f && v.x <= 1.0f && __builtin_fabsf(v.y) <= 1.0f)) return UH_ERR_RANGE;
  const float fr = __builtin_amdgcn_fractf(v.x * 0x1p30f) + __builtin_amdgcn_fractf(v.y * 0x1p30f);
  return fr == 0.0f ? 0 : UH_ERR_GRID;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Equal-x rule at the junction of two hoods (vertical closure): if P's last
// and Q's first corner share x, only the higher survives (ties: P's, which
// has the lower index).  Adjusts hp, or sets qs = 1 to skip Q's first.
__device__ __forceinline__ void junction_rule(float2 plast, float2 qfirst,
                                              int &hp, int &qs) {
  if (plast.x == qfirst.x) {
    if (qfirst.y > plast.y)
      --hp;
    else
      qs = 1;
  }
}

// Start of set s's points (and of its output slots).  A single-set run
// (both hoods: set 1 is the mirrored copy, its slots n further on) needs no
// table.
__device__ __forceinline__ int64_t set_base(const RunArgs &A, int s) {
  return A.one_set ? (int64_t)s * A.n_points : A.set_start[s];
}
__device__ __forceinline__ int64_t set_size(const RunArgs &A, int s) {
  return A.one_set ? A.n_points : A.set_start[s + 1] - A.set_start[s];
}

// Rounds of pairwise merges over a set's serial strip hoods of K points:
// ceil(log2(ceil(n / K))) (the strips themselves stand for the paper's first
// log2(K) - 1 stages, which start at blocks of two points).
__device__ __forceinline__ int32_t merge_rounds(int64_t n, int K) {
  const int64_t strips = (n + K - 1) / K;
  int32_t r = 0;
  while (((int64_t)1 << r) < strips) ++r;
  return r;
}

// The set's final writer records its status and round count in the stats.
__device__ __forceinline__ void finish_stats(const RunArgs &A, int set, int32_t status) {
  if (A.stats) {
    A.stats[set].rounds = merge_rounds(set_size(A, set), A.tile_len / 64);
    A.stats[set].status = status;
  }
}

// ---------------------------------------------------------------- init
// Also clears the first `groups` group maxima: a run in a workspace shared
// by runs of other shapes cannot rely on the previous run having left them
// zero (a plan's own workspace can: every run's final merges zero them).
__global__ void init_kernel(int32_t S, int32_t groups, RunArgs A) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < groups) {
    A.group_max[(int64_t)s * GROUP_STRIDE] = 0u;
    A.group_max[(int64_t)s * GROUP_STRIDE + 1] = 0u;  // the replicas' counter (merge_kernel)
  }
  if (s >= S) return;
  A.set_status[s] = 0;
  if (A.stats) {
    A.stats[s].orient_evals = 0;
    A.stats[s].fallbacks = 0;
    A.stats[s].sign_errors = 0;
    A.stats[s].rounds = 0;
    A.stats[s].status = 0;
  }
  if (set_size(A, s) == 0) A.out_counts[s] = 0;
}

// ---------------------------------------------------------------- tiles
// Workgroup barrier that orders LDS only: unlike __syncthreads it does not
// wait for outstanding global loads, so a prefetch stays in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- lane moves inside the VALU (DPP, GFX9 encodings); a lane whose source
// lies outside its row (or the wave) keeps `old`.
enum : int {
  DPP_ROW_SHL = 0x100,       // + n: lane i <- lane i + n of the same row of 16
  DPP_ROW_SHR = 0x110,       // + n: lane i <- lane i - n of the same row
  DPP_WAVE_SHL1 = 0x130,     // lane i <- lane i + 1
  DPP_WAVE_SHR1 = 0x138,     // lane i <- lane i - 1
  DPP_ROW_HALF_MIRROR = 0x141,
  DPP_ROW_BCAST15 = 0x142,   // lane 15 of each row -> the next row
  DPP_ROW_BCAST31 = 0x143,   // lane 31 -> rows 2 and 3
  DPP_QUAD_XOR1 = 0xB1,      // quad_perm [1, 0, 3, 2]
  DPP_QUAD_XOR2 = 0x4E,      // quad_perm [2, 3, 0, 1]
};

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v),
                                                    CTRL, ROW_MASK, 0xf, false));
}

__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Inclusive max over the lanes of each row of 16 at or below (prefix) or at
// or above (suffix) this lane; `id` is below every value.
__device__ __forceinline__ float row_prefix_max(float v, float id) {
  v = fmaxf(v, dpp<DPP_ROW_SHR + 1>(id, v));
  v = fmaxf(v, dpp<DPP_ROW_SHR + 2>(id, v));
  v = fmaxf(v, dpp<DPP_ROW_SHR + 4>(id, v));
  v = fmaxf(v, dpp<DPP_ROW_SHR + 8>(id, v));
  return v;
}
__device__ __forceinline__ float row_suffix_max(float v, float id) {
  v = fmaxf(v, dpp<DPP_ROW_SHL + 1>(id, v));
  v = fmaxf(v, dpp<DPP_ROW_SHL + 2>(id, v));
  v = fmaxf(v, dpp<DPP_ROW_SHL + 4>(id, v));
  v = fmaxf(v, dpp<DPP_ROW_SHL + 8>(id, v));
  return v;
}

// Wave-level inclusive prefix sum of an integer (lanes at or below this
// one), by DPP row shifts and row broadcasts: no trip through LDS.
__device__ __forceinline__ int wave_prefix_sum(int v) {
  const float z = __int_as_float(0);
  v += __float_as_int(dpp<DPP_ROW_SHR + 1>(z, __int_as_float(v)));
  v += __float_as_int(dpp<DPP_ROW_SHR + 2>(z, __int_as_float(v)));
  v += __float_as_int(dpp<DPP_ROW_SHR + 4>(z, __int_as_float(v)));
  v += __float_as_int(dpp<DPP_ROW_SHR + 8>(z, __int_as_float(v)));
  v += __float_as_int(dpp<DPP_ROW_BCAST15, 0xa>(z, __int_as_float(v)));  // rows 1, 3 add rows 0, 2
  v += __float_as_int(dpp<DPP_ROW_BCAST31, 0xc>(z, __int_as_float(v)));  // rows 2, 3 add rows 0-1
  return v;
}

// Wave-level inclusive max scans (prefix: lanes below; suffix: lanes above).
__device__ __forceinline__ float wave_prefix_max(float v, float id = -2.0f) {
  v = row_prefix_max(v, id);
  v = fmaxf(v, dpp<DPP_ROW_BCAST15, 0xa>(id, v));  // rows 1, 3 take rows 0, 2
  v = fmaxf(v, dpp<DPP_ROW_BCAST31, 0xc>(id, v));  // rows 2, 3 take rows 0-1
  return v;
}
__device__ __forceinline__ float wave_suffix_max(float v, float id = -2.0f) {
  v = row_suffix_max(v, id);
  // each row's total now sits in its first lane; add those of later rows
  const float t1 = readlane(v, 16), t2 = readlane(v, 32), t3 = readlane(v, 48);
  const float t23 = fmaxf(t2, t3), t123 = fmaxf(t1, t23);
  const int row = (threadIdx.x & 63) >> 4;
  return fmaxf(v, row == 0 ? t123 : row == 1 ? t23 : row == 2 ? t3 : id);
}

// Exclusive max over the lanes of this lane's segment of W lanes (W = 16:
// one row; W = 32: two rows) below it (pre) and above it (post).
template <int W>
__device__ __forceinline__ void segment_excl_max(float v, float id, float &pre, float &post) {
  const int lane = threadIdx.x & 63;
  float a = row_prefix_max(v, id), b = row_suffix_max(v, id);
  if constexpr (W == 16) {
    pre = dpp<DPP_ROW_SHR + 1>(id, a);
    post = dpp<DPP_ROW_SHL + 1>(id, b);
  } else {
    a = fmaxf(a, dpp<DPP_ROW_BCAST15, 0xa>(id, a));  // rows 1, 3 take rows 0, 2
    const float t1 = readlane(b, 16), t3 = readlane(b, 48);
    const int row = lane >> 4;
    b = fmaxf(b, row == 0 ? t1 : row == 2 ? t3 : id);
    pre = (lane & 31) == 0 ? id : dpp<DPP_WAVE_SHR1>(id, a);
    post = (lane & 31) == 31 ? id : dpp<DPP_WAVE_SHL1>(id, b);
  }
}

// Number of set bits of m in the lanes below this one.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Position of set bit k (from 0, counting up from bit 0) of m, for
// k < popcount(m): a binary search over the counts of m's lower bits.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int k) {
  int base = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const int c = __builtin_popcountll((m >> base) & ((1ull << w) - 1ull));
    if (k >= c) {
      k -= c;
      base += w;
    }
  }
  return base;
}

// The hood of the entries of nleaf leaves blk[0 .. nleaf) (start, count) in
// xy / id, in x order, at most 64 entries in all and every leaf non-empty,
// by the direct corner test: entry c is kept iff it is a corner by the
// hood's definition -- no entry at its x is higher, or as high with a lower
// index; and either no entry lies strictly left (right) of it, or it lies
// strictly above the segment from its left tangent point (of the entries
// strictly left of it, the one with the least slope to it) to its right
// tangent point (of those strictly right, the one with the greatest slope
// from it), the segment that lies highest at its x among all that span it.
// Called by all NW waves of the workgroup.  Lane c of every wave takes entry
// c; wave w scans the entries [w vk / NW, (w + 1) vk / NW) with one
// orientation test each (against the tangent point on the entry's side),
// then the waves' partial results are combined pairwise in log2(NW) rounds
// through `part` / `pfl` (NW * 64 float4 and ints of LDS that overlap
// neither xy[0 .. 64) nor id[0 .. 64)).  The tangent points are extremes of
// slopes, so any grouping of the scan reaches the extreme; when several
// collinear entries attain it, all lie on one ray from c and give the final
// test the same sign.  Wave 0 writes the corners to xy / id from 0 on, in x
// order, and blk[0] = (0, count).  Depth: vk / NW tests and log2(NW)
// combining steps, against log2(nleaf) rounds of merges.
template <int NW, class ID>
__device__ __forceinline__ void block_direct_hood(float2 *xy, ID *id, int2 *blk, int nleaf,
                                                  OrientCount &oc, bool fe, float4 *part,
                                                  int *pfl) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int2 lf = lane < nleaf ? blk[lane] : make_int2(0, 0);
  const int incl = wave_prefix_sum(lf.y);  // entries in leaves 0 .. lane
  const int vk = __builtin_amdgcn_readlane(incl, 63);
  int li = 0;  // the leaf of entry `lane`
  for (int k = 0; k < nleaf; ++k) li += __builtin_amdgcn_readlane(incl, k) <= lane ? 1 : 0;
  li = min(li, 63);
  const int excl = __shfl(incl - lf.y, li, 64), lo = __shfl(lf.x, li, 64);
  float2 cp = make_float2(0.f, 0.f);
  int ci = 0;
  if (lane < vk) {
    cp = xy[lo + lane - excl];
    ci = (int)id[lo + lane - excl];
  }
  __syncthreads();  // every entry is read before anything is written
  // Branch-free: every lane evaluates one test per entry, against the
  // tangent point on the entry's side (a lane that needs no test evaluates
  // it on its own point, an exact zero, and ignores it).
  const bool valid = lane < vk;
  bool hidden = !valid, have_l = false, have_r = false;
  float2 lt = cp, rt = cp;
  for (int e = w * vk / NW; e < (w + 1) * vk / NW; ++e) {
    const float2 q = make_float2(readlane(cp.x, e), readlane(cp.y, e));
    const int qi = __builtin_amdgcn_readlane(ci, e);
    const bool same = q.x == cp.x, left = q.x < cp.x;
    const bool have = left ? have_l : have_r;
    // left: q replaces lt if strictly left of lt -> c; right: rt if
    // strictly left of c -> rt
    const float2 u = left ? lt : cp, v = left ? cp : rt;
    const int sg = orient_sign(u, v, q, oc, fe, valid & !same & have);
    const bool take = !same & (!have | (sg > 0));
    hidden = hidden | (same & ((q.y > cp.y) | ((q.y == cp.y) & (qi < ci))));
    lt = (take & left) ? q : lt;
    rt = (take & !left) ? q : rt;
    have_l = have_l | (!same & left);
    have_r = have_r | (!same & !left);
  }
#pragma unroll
  for (int st = 1; st < NW; st <<= 1) {  // wave w takes wave w + st's partial result
    if ((w & (2 * st - 1)) == st) {
      part[w * 64 + lane] = make_float4(lt.x, lt.y, rt.x, rt.y);
      pfl[w * 64 + lane] = (hidden ? 1 : 0) | (have_l ? 2 : 0) | (have_r ? 4 : 0);
    }
    __syncthreads();
    if ((w & (2 * st - 1)) == 0) {
      const float4 o = part[(w + st) * 64 + lane];
      const int f = pfl[(w + st) * 64 + lane];
      const float2 ol = make_float2(o.x, o.y), orr = make_float2(o.z, o.w);
      const bool ohl = (f & 2) != 0, ohr = (f & 4) != 0;
      hidden = hidden | ((f & 1) != 0);
      const int sl = orient_sign(lt, cp, ol, oc, fe, valid & have_l & ohl);
      lt = (ohl & (!have_l | (sl > 0))) ? ol : lt;
      have_l = have_l | ohl;
      const int sr = orient_sign(cp, rt, orr, oc, fe, valid & have_r & ohr);
      rt = (ohr & (!have_r | (sr > 0))) ? orr : rt;
      have_r = have_r | ohr;
    }
  }
  if (w == 0) {
    const bool spans = !hidden & have_l & have_r;
    const int sc = orient_sign(lt, rt, cp, oc, fe, spans);
    const bool corner = !hidden & (!spans | (sc > 0));
    const uint64_t cm = __ballot(corner);
    if (corner) {
      const int r = lanes_below(cm);
      xy[r] = cp;
      id[r] = (ID)ci;
    }
    if (lane == 0) blk[0] = make_int2(0, __builtin_popcountll(cm));
  }
}

// Adds a wave's orientation counters to stats[set].
__device__ __forceinline__ void flush_wave_stats(const RunArgs &A, int set, OrientCount &oc) {
  if (!A.stats) return;
  const uint32_t e = wave_sum(oc.evals), f = wave_sum(oc.fallbacks);
  const uint32_t x = wave_sum(oc.sign_errors);
  if ((threadIdx.x & 63) == 0 && A.stats && e) {
    atomicAdd((unsigned long long *)&A.stats[set].orient_evals, (unsigned long long)e);
    atomicAdd((unsigned long long *)&A.stats[set].fallbacks, (unsigned long long)f);
    if (x) atomicAdd((unsigned long long *)&A.stats[set].sign_errors, (unsigned long long)x);
  }
  oc.evals = oc.fallbacks = oc.sign_errors = 0;
}

// The counters of a kernel of this run (soundness check on request).
__device__ __forceinline__ OrientCount run_counter(const RunArgs &A) {
  OrientCount oc;
  oc.check = (A.flags & UH_FLAG_CHECK_SIGNS) != 0;
  return oc;
}

// Order-preserving unsigned code of a float (larger float, larger code;
// every code is positive, so 0 means "no value").
__device__ __forceinline__ uint32_t y_code(float y) {
  const uint32_t b = __float_as_uint(y);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float y_decode(uint32_t c) {
  if (c == 0u) return -2.0f;  // below every valid y
  return __uint_as_float((c & 0x80000000u) ? (c & 0x7fffffffu) : ~c);
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// Tile kernel: one wave (one workgroup of 64 lanes) per tile of up to
// T = 64 * K points of one set; no workgroup barrier anywhere.
//  1. coalesced 16-byte loads (two points per lane per load) and the data
//     contract's checks, then the points go to per-lane strips of K
//     consecutive points in LDS (swizzled 16-byte chunks, no padding) and
//     each lane reads its strip back into registers.  A partial tile is
//     padded with points right of and below every valid point, which no
//     test keeps;
//  2. strip pass 1: x non-decreasing check (the previous strip's last point
//     comes from the neighbouring lane), maximum y of each strip; wave
//     prefix and suffix maxima over the strips;
//  3. exact elimination.  A point r is dropped when some earlier point of
//     the set is at least as high and some later point is strictly higher:
//     r then lies below the segment joining the first earlier maximum and
//     the last later maximum (both of which survive), or directly below a
//     point at its x, so it is no corner of the hood (nor is any identical
//     copy of it that survives only because it comes later).  Witnesses are
//     the tile's points and 16 points on either side of it.  Only a strip
//     whose maximum beats every earlier strip, or reaches the maximum of
//     every later one, can hold a survivor; with strips of 16, four such
//     strips at a time are tested point by point by the 16 lanes of one
//     row each.  Few survivors go out as a sorted point list (the merge
//     kernel makes it a hood); otherwise
//  4. the survivors of each strip go through a serial monotone chain whose
//     stack lives in the strip's LDS slot (the serial strip hoods of the
//     paper's work-optimal variant), then up to six rounds of Wagener merges
//     (match-and-merge on adjacent hoods), the 2^(j+1) lanes of each merge
//     acting as the paper's d1 x d2 thread block;
//  5. the tile's hood goes to the workspace, or to the output for a
//     one-tile set.
// With BOTH, steps 2-5 run a second time on the same registers with every
// y negated: the lower hood is the upper hood of the mirrored points.  Its
// results go to the mirrored set (set + lower_sets, slots + lower_n, tile +
// lower_tiles, group + lower_groups), so the points are read once for both.

// 16-byte chunk c of strip s sits at chunk c ^ tile_swz<K>(s) of the slot,
// so the transpose writes (8 lanes per strip) and the strip reads (one strip
// per lane) touch distinct LDS banks.
template <int K>
__device__ __forceinline__ int tile_swz(int strip) {
  return (strip ^ (strip >> 3)) & (K / 2 - 1);
}

constexpr float TILE_PAD_X = 2.0f, TILE_PAD_Y = -4.0f;  // right of / below every valid point

// Steps 2 (maxima) to 5 of one hood of the tile whose points are p (this
// lane's strip, in registers) and, transposed, in sxy.  nb_before / nb_after:
// highest y of the witnesses before / after the tile (-2: none); err: the
// tile's data status.
template <int K>
__device__ __forceinline__ void tile_hood(const RunArgs &A, const TileItem &it, int tile,
                                          int32_t *cnt_out, const float2 (&p)[K],
                                          float nb_before, float nb_after, float2 set_first,
                                          float2 set_last, int err, bool fe,
                                          float2 *sxy, uint16_t *sid) {
  constexpr int S = K;
  const int lane = threadIdx.x;
  const bool fin = it.rel0 == 0 && it.len == it.set_len;  // the set's only tile
  float2 *st = sxy + lane * S;
  uint16_t *sl = sid + lane * S;
  OrientCount oc = run_counter(A);
  float ymax = TILE_PAD_Y;
#pragma unroll
  for (int i = 0; i < K; ++i) ymax = fmaxf(ymax, p[i].y);
  const float incp = wave_prefix_max(ymax), incs = wave_suffix_max(ymax);
  {
    // the tile's highest point: a witness for the first merge level
    const uint32_t code = y_code(readlane(incp, 63));
    if (it.group >= 0 && lane == 0) {
      A.tile_max[tile] = code;
      atomicMax(&A.group_max[it.group * GROUP_STRIDE], code);
    }
  }
  const float exp_pre = fmaxf(dpp<DPP_WAVE_SHR1>(-2.0f, incp), nb_before);  // earlier strips
  const float exp_suf = fmaxf(dpp<DPP_WAVE_SHL1>(-2.0f, incs), nb_after);   // later strips
  const int rel0 = it.rel0;

  // ---- 3. elimination; few survivors leave as a point list
  // Without elimination (UH_FLAG_NO_ELIMINATION) every point of the tile
  // goes through the strip hoods and the rounds, and the tile leaves a hood.
  const bool noelim = (A.flags & UH_FLAG_NO_ELIMINATION) != 0;
  if ((K == 16 || K == 32) && !fin && !noelim) {
    constexpr int SPP = 64 / K;  // candidate strips per pass
    const uint64_t cand = __ballot(ymax > exp_pre || ymax >= exp_suf);
    const int ncand = __builtin_popcountll(cand);
    if (ncand <= 4 * SPP) {
      // each segment of K lanes takes one candidate strip per pass; lane i of
      // the segment tests point i against the exact earlier / later maxima
      const int seg = lane / K, i = lane % K;
      const int npass = (ncand + SPP - 1) / SPP;
      uint64_t rest = cand, kb[4];
      float2 kp[4];
      int kid[4], nsurv = 0;
#pragma unroll
      for (int ps = 0; ps < 4; ++ps) {
        kb[ps] = 0;
        kp[ps] = make_float2(0.f, 0.f);
        kid[ps] = 0;
        if (ps < npass) {
          int Ls[SPP];
#pragma unroll
          for (int rr = 0; rr < SPP; ++rr) {
            Ls[rr] = rest ? (int)__builtin_ctzll(rest) : -1;
            rest &= rest - 1;
          }
          int L = Ls[0];
#pragma unroll
          for (int rr = 1; rr < SPP; ++rr) L = seg == rr ? Ls[rr] : L;
          const int Lc = L < 0 ? 0 : L;
          const float2 q = sxy[Lc * S + 2 * ((i >> 1) ^ tile_swz<K>(Lc)) + (i & 1)];
          const float2 w = make_float2(__shfl(exp_pre, Lc, 64), __shfl(exp_suf, Lc, 64));
          float in_pre, in_post;
          segment_excl_max<K == 32 ? 32 : 16>(q.y, -2.0f, in_pre, in_post);
          const float before = fmaxf(w.x, in_pre);
          const float after = fmaxf(w.y, in_post);
          const bool keep = L >= 0 && (q.y > before || q.y >= after);
          kb[ps] = __ballot(keep);
          kp[ps] = q;
          kid[ps] = Lc * K + i;
          nsurv += __builtin_popcountll(kb[ps]);
        }
      }
      if (nsurv <= TILE_LIST_MAX) {
        int base = 0;
#pragma unroll
        for (int ps = 0; ps < 4; ++ps) {
          if ((kb[ps] >> lane) & 1ull) {
            const int r = base + lanes_below(kb[ps]);
            A.ws_xy[it.start + r] = kp[ps];
            A.ws_idx[it.start + r] = rel0 + kid[ps];
          }
          base += __builtin_popcountll(kb[ps]);
        }
        if (lane == 0) cnt_out[tile] = (int)((uint32_t)nsurv | POINTS_FLAG);
        if (err) atomicMin(&A.set_status[it.set], err);
        return;
      }
    }
  }
  uint32_t keep = 0;
  if (noelim) {
    const int my_len = min(max(it.len - lane * K, 0), K);
    keep = my_len >= 32 ? ~0u : (1u << my_len) - 1u;
  } else {
    float bm = exp_pre;  // max y over earlier points of the set
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (p[i].y > bm || p[i].y >= exp_suf) keep |= 1u << i;
      bm = fmaxf(bm, p[i].y);
    }
  }
  // Chord tests: a point strictly between two points a and b of its set in x
  // that lies on or below the segment a b is no corner (the hood's
  // definition).  They catch what the height test above cannot: the points
  // of a convex arm, and the lower hood of an arch.  Pairs: the set's first
  // and last points, then the tile's.  Each is worth its orientation tests
  // only where strips lie below it: each lane first estimates (in plain
  // float32, a guess that decides nothing but whether to test) on which side
  // the first point of its strip lies, and the tile runs the exact test if
  // 48 lanes find theirs below (not on the noise of a nearly straight run).
  bool chord_ran = false, nb_ran = false;
  if (!noelim) {
    const int ll = it.len - 1, lane_l = ll / K, il = ll % K;
    const float2 tf = make_float2(readlane(p[0].x, 0), readlane(p[0].y, 0));
    const float2 tl = sxy[lane_l * S + 2 * ((il >> 1) ^ tile_swz<K>(lane_l)) + (il & 1)];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float2 f = c == 0 ? set_first : tf, l = c == 0 ? set_last : tl;
      const float est = (l.x - f.x) * (p[0].y - f.y) - (l.y - f.y) * (p[0].x - f.x);
      const bool below0 = lane * K < it.len && est < 0.0f;
      if (__builtin_popcountll(__ballot(below0)) >= 48) {
        chord_ran = true;
#pragma unroll
        for (int i = 0; i < K; ++i)
          if (((keep >> i) & 1u) && f.x < p[i].x && p[i].x < l.x &&
              orient_sign(f, l, p[i], oc, fe) <= 0)
            keep &= ~(1u << i);
      }
    }
    // Neighbour chords: the points of each strip against the segment joining
    // a point of the strip before it and a point of the strip after it (real
    // points of the set; tested only for points strictly between them in x).
    // Seen at the scale of a strip, a hull-heavy arc or parabola is a nearly
    // straight run of noisy points.  Each strip offers as its witness the
    // point highest above the local direction of the run (the line through
    // the first points of its two neighbouring strips): such points lie at
    // the top of the noise, and most of the strip between two of them lies
    // under their segment.  The choice is a float32 guess (any real point is
    // a valid witness); the test drops a point only where the FP32 filter
    // certifies it strictly below the segment, and keeps it otherwise.  On a
    // strongly curved run the strip lies above the segment and the tile
    // skips the test (the same float32 guess as above, 16 lanes).
    {
      const int my_n = min(max(it.len - lane * K, 0), K);
      const float dxs = dpp<DPP_WAVE_SHL1>(p[0].x, p[0].x) - dpp<DPP_WAVE_SHR1>(p[0].x, p[0].x);
      const float dys = dpp<DPP_WAVE_SHL1>(p[0].y, p[0].y) - dpp<DPP_WAVE_SHR1>(p[0].y, p[0].y);
      float2 m = p[0];
      float best = p[0].y * dxs - p[0].x * dys;
#pragma unroll
      for (int i = 1; i < K; ++i) {
        const float sc = p[i].y * dxs - p[i].x * dys;
        if (i < my_n && sc > best) {
          best = sc;
          m = p[i];
        }
      }
      const float2 ma = make_float2(dpp<DPP_WAVE_SHR1>(0.0f, m.x), dpp<DPP_WAVE_SHR1>(0.0f, m.y));
      const float2 mb = make_float2(dpp<DPP_WAVE_SHL1>(0.0f, m.x), dpp<DPP_WAVE_SHL1>(0.0f, m.y));
      const bool nb_ok = lane >= 1 && lane <= 62 && (lane + 1) * K < it.len;
      const float est = (mb.x - ma.x) * (p[0].y - ma.y) - (mb.y - ma.y) * (p[0].x - ma.x);
      if (__builtin_popcountll(__ballot(nb_ok && est < 0.0f)) >= 16) {
        nb_ran = true;
        if (nb_ok) {
#pragma unroll
          for (int i = 0; i < K; ++i)
            if (((keep >> i) & 1u) && ma.x < p[i].x && p[i].x < mb.x &&
                surely_below(ma, mb, p[i], oc, fe))
              keep &= ~(1u << i);
        }
      }
    }
  }
  // After the neighbour chords the points left are few per strip but not
  // few per tile (hull-heavy data): they go through the strip hoods and
  // rounds below rather than to the merge kernel's serial chain.
  if (((K != 16 && K != 32) || chord_ran) && !noelim && !nb_ran) {
    // few survivors leave as a sorted point list: ranks by a wave prefix sum
    // (with strips of 16 or 32 the height test's survivors were counted
    // already; only the chord tests can have left few)
    const int nk = __builtin_popcount(keep);
    int koff = wave_prefix_sum(nk);
    const int nsurv = __shfl(koff, 63, 64);
    koff -= nk;
    if (!fin && nsurv <= TILE_LIST_MAX) {
      int r = koff;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        if ((keep >> i) & 1u) {
          A.ws_xy[it.start + r] = p[i];
          A.ws_idx[it.start + r] = rel0 + lane * K + i;
          ++r;
        }
      }
      if (lane == 0) cnt_out[tile] = (int)((uint32_t)nsurv | POINTS_FLAG);
      if (err) atomicMin(&A.set_status[it.set], err);
      flush_wave_stats(A, it.set, oc);
      return;
    }
  }

  // ---- 4. strip hoods, then rounds of Wagener merges over them
  int nleaf;
  int2 leaf = make_int2(0, 0);  // lane l: leaf l (base, count)
  if (!noelim) {
    // After the eliminations most strips keep a point or two: serial hoods
    // of whole strips would leave up to 64 tiny leaves and six rounds of
    // merges.  The survivors are compacted instead, in x order, into the
    // LDS arrays (the strips' points are in registers by now) and cut into
    // chunks of C consecutive survivors; lane l builds the serial hood of
    // chunk l in place (the serial hoods of the work-optimal variant's
    // strips, over survivors rather than over all points).  The chunk hoods
    // are the leaves: every chunk keeps at least one corner.
    const int nk = __builtin_popcount(keep);
    int koff = wave_prefix_sum(nk);
    const int nsurv = __shfl(koff, 63, 64);
    koff -= nk;
    wave_sync();  // every lane is done with the strips in LDS
    {
      int r = koff;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        if ((keep >> i) & 1u) {
          sxy[r] = p[i];
          sid[r] = (uint16_t)(lane * K + i);
          ++r;
        }
      }
    }
    wave_sync();
    int C = 8;  // chunk length: at most 64 chunks
    while (C * 64 < nsurv) C <<= 1;
    nleaf = (nsurv + C - 1) / C;
    if (lane < nleaf) {
      const int b = lane * C;
      leaf = make_int2(b, chain_inplace(sxy + b, sid + b, min(C, nsurv - b), oc, fe));
    }
    wave_sync();
  } else {
    // the serial strip hood over each strip's survivors, taken from the
    // registers in order; its stack overwrites the strip's LDS slot from
    // the start (in plain order); the non-empty strip hoods are the leaves
    int cnt = 0;
    float2 t1 = make_float2(0.f, 0.f), t2 = t1;  // stack top, second
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (!((keep >> i) & 1u)) continue;
      const float2 r = p[i];
      if (cnt >= 1 && r.x == t1.x) {
        if (r.y <= t1.y) continue;  // the top hides r (ties: lower index)
        --cnt;                      // r hides the top
        t1 = t2;
        if (cnt >= 2) t2 = st[cnt - 2];
      }
      while (cnt >= 2 && orient_sign(t2, t1, r, oc, fe) >= 0) {
        --cnt;  // the top is on or below t2 -> r
        t1 = t2;
        if (cnt >= 2) t2 = st[cnt - 2];
      }
      st[cnt] = r;
      sl[cnt] = (uint16_t)(lane * K + i);
      t2 = t1;
      t1 = r;
      ++cnt;
    }
    // Nothing between two consecutive leaves survived, so merging
    // neighbouring leaves is merging hoods of x-adjacent point sets.
    const uint64_t ne = __ballot(cnt > 0);
    nleaf = __builtin_popcountll(ne);
    const int src = lane < nleaf ? nth_set_bit(ne, lane) : 0;  // the strip of leaf `lane`
    const int csrc = __shfl(cnt, src, 64);
    if (lane < nleaf) leaf = make_int2(src * S, csrc);
    wave_sync();
  }
  leaf = wave_rounds(sxy, sid, leaf, nleaf, oc, fe);

  // ---- 5. output
  const int hb = nleaf ? leaf.x : 0, hc = nleaf ? leaf.y : 0;
  if (fin) {
    if (__ballot(err != 0)) err = wave_min(err);
    int32_t *dst = A.out_idx + (it.start - it.rel0);
    for (int k = lane; k < hc; k += 64) dst[k] = rel0 + (int)sid[hb + k];
    if (lane == 0) {
      A.out_counts[it.set] = err ? err : hc;
      finish_stats(A, it.set, err);
    }
  } else {
    for (int k = lane; k < hc; k += 64) {
      A.ws_xy[it.start + k] = sxy[hb + k];
      A.ws_idx[it.start + k] = rel0 + (int)sid[hb + k];
    }
    if (lane == 0) cnt_out[tile] = hc;
    if (err) atomicMin(&A.set_status[it.set], err);
  }
  flush_wave_stats(A, it.set, oc);
}

// The tile a wave works on: from the table, or in a single-set run from
// its index (tile t of the only set, ntiles tiles in all).
__device__ __forceinline__ TileItem tile_item(const RunArgs &A, const TileItem *items, int tile,
                                              int ntiles) {
  TileItem it;
  if (A.one_set) {
    it.start = (int64_t)tile * A.tile_len;
    it.len = (int32_t)min((int64_t)A.tile_len, A.n_points - it.start);
    it.set = 0;
    it.rel0 = (int32_t)it.start;
    it.nb_lo = (int16_t)min(16, it.rel0);
    it.nb_hi = (int16_t)min((int64_t)16, A.n_points - it.start - it.len);
    it.set_len = (int32_t)A.n_points;
    it.group = ntiles == 1 ? -1 : tile / A.group_fan;
  } else {
    it = items[tile];
  }
  return it;
}

// Everything a tile reads from global memory: its points (a partial tile
// padded with points right of and below every valid point), up to 16
// witness points on either side of it (lanes 0-15, two each: their y), the
// set's first and last point and the set's point just before the tile.
template <int K>
struct TileLoad {
  float4 v[K / 2];
  float y0, y1;
  float2 set_first, set_last;
  float prev_x;
};

// Issues every load of tile `it` without waiting for any of them.
template <int K>
__device__ __forceinline__ void tile_load(const RunArgs &A, const TileItem &it, TileLoad<K> &L) {
  constexpr int NV = K / 2;
  constexpr float PAD_X = TILE_PAD_X, PAD_Y = TILE_PAD_Y;
  const int lane = threadIdx.x;
  const float2 *src = A.pts + it.start;
  const bool full = it.len == 64 * K && (((uintptr_t)src) & 15u) == 0;
  if (full) {
    // full, 16-byte aligned tile (the common case): no per-element tests
    const float4 *src4 = reinterpret_cast<const float4 *>(__builtin_assume_aligned(src, 16));
#pragma unroll
    for (int r = 0; r < NV; ++r) L.v[r] = src4[lane + 64 * r];
  } else {
    const bool al = (((uintptr_t)src) & 15u) == 0;
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int e = 2 * (lane + 64 * r);
      L.v[r] = make_float4(PAD_X, PAD_Y, PAD_X, PAD_Y);
      if (e + 1 < it.len) {
        if (al) {
          L.v[r] = *reinterpret_cast<const float4 *>(src + e);
        } else {
          const float2 a = src[e], b = src[e + 1];
          L.v[r] = make_float4(a.x, a.y, b.x, b.y);
        }
      } else if (e < it.len) {
        const float2 a = src[e];
        L.v[r].x = a.x;
        L.v[r].y = a.y;
      }
    }
  }
  // witnesses: unconditionally, at clamped addresses
  const int64_t wlo = it.start - it.nb_lo, whi = it.start + it.len + it.nb_hi;
  const int64_t e = lane < 8 ? it.start - 16 + 2 * lane : it.start + it.len + 2 * (lane - 8);
  const bool ok0 = lane < 16 && (lane < 8 ? e >= wlo : e < whi);
  const bool ok1 = lane < 16 && (lane < 8 ? e + 1 >= wlo : e + 1 < whi);
  L.y0 = A.pts[ok0 ? e : it.start].y;
  L.y1 = A.pts[ok1 ? e + 1 : it.start].y;
  const int64_t set0 = it.start - it.rel0;
  L.set_first = A.pts[set0];
  L.set_last = A.pts[set0 + it.set_len - 1];
  L.prev_x = A.pts[it.start - (it.rel0 > 0 ? 1 : 0)].x;
}

// Steps 1 (checks, strips) to 5 of one tile whose loads are in L.
template <int K, bool BOTH>
__device__ __forceinline__ void tile_process(const RunArgs &A, const TileItem &it, int tile,
                                             int32_t *cnt_out, const TileLoad<K> &L,
                                             float2 *sxy, uint16_t *sid) {
  constexpr int S = K;       // a strip's slot in LDS: K points, no padding
  constexpr int NV = K / 2;  // 16-byte slots (point pairs) per lane
  const int lane = threadIdx.x;
  const bool fe = (A.flags & UH_FLAG_FORCE_FALLBACK) != 0;
  const bool validate = (A.flags & UH_FLAG_NO_VALIDATE) == 0;
  const float2 *src = A.pts + it.start;
  const bool full = it.len == 64 * K && (((uintptr_t)src) & 15u) == 0;
  float4 v[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) v[r] = L.v[r];
  float w0, w1;  // this lane's two witness heights (-2: none)
  float m0 = -2.0f, m1 = -2.0f;  // ... mirrored, for the lower hood
  {
    const int64_t wlo = it.start - it.nb_lo, whi = it.start + it.len + it.nb_hi;
    const int64_t e = lane < 8 ? it.start - 16 + 2 * lane : it.start + it.len + 2 * (lane - 8);
    const bool ok0 = lane < 16 && (lane < 8 ? e >= wlo : e < whi);
    const bool ok1 = lane < 16 && (lane < 8 ? e + 1 >= wlo : e + 1 < whi);
    w0 = ok0 ? L.y0 : -2.0f;
    w1 = ok1 ? L.y1 : -2.0f;
    if constexpr (BOTH) {
      m0 = ok0 ? -L.y0 : -2.0f;
      m1 = ok1 ? -L.y1 : -2.0f;
    }
  }
  float2 set_first = L.set_first, set_last = L.set_last;  // chord of the set
  const float prev_tile_x = validate && it.rel0 > 0 ? L.prev_x : -1.0f;  // -1: below every valid x

  int err = 0;
  bool bad = false;  // some check failed, or the quick checks cannot vouch
  if (full) {
    if (validate) {
      // Quick checks that can only err towards `bad`: |y| <= 1 (NaN fails
      // the grid test instead), y * 2^30 without fraction (the bits of a
      // zero fraction are zero), x within [0, 1] at the tile's ends (the
      // strip pass checks x non-decreasing, NaN included), and x on the grid:
      // if the first x is at least 2^-7, every x is, and float32 spacing
      // there is at least 2^-30.
      float ry = 0.0f;
      uint32_t gy = 0u;
#pragma unroll
      for (int r = 0; r < NV; ++r) {
        ry = fmaxf(ry, fmaxf(__builtin_fabsf(v[r].y), __builtin_fabsf(v[r].w)));
        gy |= __float_as_uint(__builtin_amdgcn_fractf(v[r].y * 0x1p30f)) |
              __float_as_uint(__builtin_amdgcn_fractf(v[r].w * 0x1p30f));
      }
      const float x_first = readlane(v[0].x, 0), x_last = readlane(v[NV - 1].z, 63);
      bad = !(ry <= 1.0f) || gy != 0u || !(x_first >= 0.0f) || !(x_last <= 1.0f);
      if (!(x_first >= 0x1p-7f)) {
        uint32_t gx = 0u;
#pragma unroll
        for (int r = 0; r < NV; ++r)
          gx |= __float_as_uint(__builtin_amdgcn_fractf(v[r].x * 0x1p30f)) |
                __float_as_uint(__builtin_amdgcn_fractf(v[r].z * 0x1p30f));
        bad = bad || gx != 0u;
      }
    }
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int e = 2 * (lane + 64 * r);
      float4 *d = reinterpret_cast<float4 *>(__builtin_assume_aligned(
          sxy + (e / K) * S + 2 * (((e % K) >> 1) ^ tile_swz<K>(e / K)), 16));
      *d = v[r];
    }
  } else {
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int e = 2 * (lane + 64 * r);
      if (validate) {
        if (e < it.len) err = min(err, check_point(make_float2(v[r].x, v[r].y)));
        if (e + 1 < it.len) err = min(err, check_point(make_float2(v[r].z, v[r].w)));
      }
      *reinterpret_cast<float4 *>(sxy + (e / K) * S + 2 * (((e % K) >> 1) ^ tile_swz<K>(e / K))) =
          v[r];
    }
    bad = err != 0;
  }
  // witness maxima: over each group of 8 lanes, then read from lanes 0 and 8
  float nb_before, nb_after, mb_before = -2.0f, mb_after = -2.0f;
  {
    float wy = fmaxf(w0, w1);
    wy = fmaxf(wy, dpp<DPP_QUAD_XOR1>(wy, wy));
    wy = fmaxf(wy, dpp<DPP_QUAD_XOR2>(wy, wy));
    wy = fmaxf(wy, dpp<DPP_ROW_HALF_MIRROR>(wy, wy));
    nb_before = readlane(wy, 0);
    nb_after = readlane(wy, 8);
    if constexpr (BOTH) {
      float my = fmaxf(m0, m1);
      my = fmaxf(my, dpp<DPP_QUAD_XOR1>(my, my));
      my = fmaxf(my, dpp<DPP_QUAD_XOR2>(my, my));
      my = fmaxf(my, dpp<DPP_ROW_HALF_MIRROR>(my, my));
      mb_before = readlane(my, 0);
      mb_after = readlane(my, 8);
    }
  }
  wave_sync();
  const int my_len = min(max(it.len - lane * K, 0), K);
  float2 *st = sxy + lane * S;
  float2 p[K];
#pragma unroll
  for (int k = 0; k < K / 2; ++k) {
    const float4 q = *reinterpret_cast<const float4 *>(st + 2 * (k ^ tile_swz<K>(lane)));
    p[2 * k] = make_float2(q.x, q.y);
    p[2 * k + 1] = make_float2(q.z, q.w);
  }

  // ---- 2. strip pass 1: x order (the last point of the previous strip;
  // lane 0: of the previous tile)
  {
    const float px0 = dpp<DPP_WAVE_SHR1>(prev_tile_x, p[K - 1].x);
    float px = px0;
    bool uns = false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      uns = uns || !(p[i].x >= px);
      px = p[i].x;
    }
    if (validate && __ballot(bad || uns)) {
      // something is off in this tile: the exact error codes, point by point
      err = 0;
      px = px0;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        if (i < my_len) {
          err = min(err, check_point(p[i]));
          if (p[i].x < px) err = min(err, UH_ERR_UNSORTED);
          px = p[i].x;
        }
      }
    }
  }
  tile_hood<K>(A, it, tile, cnt_out, p, nb_before, nb_after, set_first, set_last, err, fe, sxy,
               sid);

  if constexpr (BOTH) {
    // the lower hood: the same points mirrored in the x axis (the padding
    // stays below every valid point), back in their LDS strips
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (i < my_len) p[i].y = -p[i].y;
    wave_sync();  // every lane is done with the upper hood's LDS
#pragma unroll
    for (int k = 0; k < K / 2; ++k)
      *reinterpret_cast<float4 *>(st + 2 * (k ^ tile_swz<K>(lane))) =
          make_float4(p[2 * k].x, p[2 * k].y, p[2 * k + 1].x, p[2 * k + 1].y);
    wave_sync();
    TileItem lo = it;
    lo.start += A.lower_n;
    lo.set += A.lower_sets;
    if (lo.group >= 0) lo.group += A.lower_groups;
    set_first.y = -set_first.y;
    set_last.y = -set_last.y;
    tile_hood<K>(A, lo, tile + A.lower_tiles, cnt_out, p, mb_before, mb_after, set_first,
                 set_last, err, fe, sxy, sid);
  }
}

// The tile pass: one wave per tile.
template <int K, bool BOTH>
__global__ __launch_bounds__(64) void tile_kernel(RunArgs A, const TileItem *items,
                                                  int32_t *cnt_out, int32_t ntiles) {
  // 10 KB at K = 16: sixteen waves per compute unit (the leaf table of the
  // in-wave rounds lives in registers)
  __shared__ __attribute__((aligned(16))) float2 sxy[64 * K];
  __shared__ uint16_t sid[64 * K];

  const int tile = blockIdx.x;
  const TileItem it = tile_item(A, items, tile, ntiles);
  TileLoad<K> ld;
  tile_load<K>(A, it, ld);
  tile_process<K, BOTH>(A, it, tile, cnt_out, ld, sxy, sid);
}

// ---------------------------------------------------------------- merges
// Exclusive prefix sum of one value per thread over the workgroup.
template <int BLK>
__device__ __forceinline__ int block_exclusive_scan(int v, int *swave, int &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int x = wave_prefix_sum(v);
  if (lane == 63) swave[w] = x;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int k = 0; k < BLK / 64; ++k) {
    if (k < w) before += swave[k];
    total += swave[k];
  }
  return before + x - v;
}

// Workgroup-wide exclusive maxima of v: over the threads below (pre) and
// above (post) this one, each also at least the maximum of `all_pre` /
// `all_post` over every thread of the workgroup.
template <int BLK>
__device__ __forceinline__ void block_excl_max(float v, float all_pre, float all_post,
                                               float &pre, float &post, float4 *sw) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const float incp = wave_prefix_max(v), incs = wave_suffix_max(v);
  const float ap = readlane(wave_prefix_max(all_pre), 63);
  const float aq = readlane(wave_prefix_max(all_post), 63);
  if (lane == 0) sw[w] = make_float4(readlane(incp, 63), readlane(incs, 0), ap, aq);
  pre = dpp<DPP_WAVE_SHR1>(-2.0f, incp);
  post = dpp<DPP_WAVE_SHL1>(-2.0f, incs);
  __syncthreads();
  for (int k = 0; k < BLK / 64; ++k) {
    const float4 q = sw[k];
    if (k < w) pre = fmaxf(pre, q.x);
    if (k > w) post = fmaxf(post, q.y);
    pre = fmaxf(pre, q.z);
    post = fmaxf(post, q.w);
  }
  __syncthreads();  // sw may be reused
}

// Segmented exclusive scan over the threads of a workgroup, in thread order:
// thread t brings (head, v), head meaning that a segment starts inside its
// chunk (v then covers only its chunk after the last start).  Returns the
// combination by op of the earlier threads' values back to the nearest start
// (ident if none); meaningful for a thread whose chunk continues a segment.
template <int BLK, class T, class OP>
__device__ __forceinline__ T seg_excl_scan(bool head, T v, T ident, OP op, T *sv, int *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  bool h = head;
  T x = v;
  for (int o = 1; o < 64; o <<= 1) {  // inclusive, within the wave
    const T x2 = __shfl_up(x, o, 64);
    const bool h2 = __shfl_up((int)h, o, 64) != 0;
    if (lane >= o) {
      x = h ? x : op(x2, x);
      h = h || h2;
    }
  }
  if (lane == 63) {
    sv[w] = x;
    sh[w] = h;
  }
  __syncthreads();
  T carry = ident;  // earlier waves, back to the nearest start
  for (int q = 0; q < w; ++q) carry = sh[q] ? sv[q] : op(carry, sv[q]);
  __syncthreads();  // sv, sh may be reused
  T xe = __shfl_up(x, 1, 64);  // exclusive within the wave
  bool he = __shfl_up((int)h, 1, 64) != 0;
  if (lane == 0) {
    xe = ident;
    he = false;
  }
  return he ? xe : op(carry, xe);
}

// The child whose entries [soff[k], soff[k + 1]) hold entry e (0 <= e < the
// total): the largest k < n with soff[k] <= e (soff is non-decreasing).
template <int BLK>
__device__ __forceinline__ int child_of(const int *soff, int n, int e) {
  int l = 0, h = n;
  while (h - l > 1) {
    const int mid = (l + h) >> 1;
    if (soff[mid] <= e) l = mid;
    else h = mid;
  }
  return l;
}

// Four consecutive 32-bit or 8-byte elements moved as one access where the
// four lie together (only 4-byte / 8-byte alignment is assumed: global
// memory accepts such wide accesses unaligned).
struct __attribute__((aligned(4))) Idx4 {
  int32_t v[4];
};
struct __attribute__((aligned(8))) Xy4 {
  float2 v[4];
};

// A block of the merge kernel's global path: children k0 .. k1 - 1, child k
// keeping corners [lo[k], lo[k] + cum[k + 1] - cum[k]) of its slot; element
// e of the block is element c0 + e of the item (cum: exclusive prefix of the
// kept counts over the item's children, in LDS).
// With lbase, the children's corner positions are also copied to LDS, child
// k's from lxy[lbase[k]] on, and the searches read them there.
struct Rope {
  const float2 *xy;
  const int *cum, *lo;
  int64_t off, stride;
  int k0, k1, c0;
  const float2 *lxy = nullptr;
  const int *lbase = nullptr;
  // The first and the last child, where the searches next to the junction
  // read: ranks below f_end are in child k0 at position f_pos + rank, ranks
  // from l_beg on in child k1 - 1 at l_pos + rank (set by prep()).
  int f_end = 0, l_beg = INT32_MAX;
  int64_t f_pos = 0, l_pos = 0;
  // the child holding the item's element gi (cum[k0] <= gi < cum[k1])
  __device__ __forceinline__ int child(int gi) const {
    int l = k0, h = k1;
    while (h - l > 1) {
      const int mid = (l + h) >> 1;
      if (cum[mid] <= gi) l = mid;
      else h = mid;
    }
    return l;
  }
  // position of child l's element of rank gi: in the workspace, or in the
  // LDS copy
  __device__ __forceinline__ int64_t pos(int l, int gi) const {
    return (lxy ? (int64_t)lbase[l] : off + (int64_t)l * stride) + lo[l] + (gi - cum[l]);
  }
  __device__ __forceinline__ void prep() {
    f_end = cum[k0 + 1];
    f_pos = pos(k0, 0);
    l_beg = cum[k1 - 1];
    l_pos = pos(k1 - 1, 0);
  }
  __device__ __forceinline__ float2 operator[](int e) const {
    const int gi = c0 + e;
    const int64_t p = gi < f_end ? f_pos + gi : gi >= l_beg ? l_pos + gi : pos(child(gi), gi);
    return lxy ? lxy[p] : xy[p];
  }
};

// Merge item b of a pass: from the table, or in a single-set run from the
// pass's shape (item i of set v).
__device__ __forceinline__ MergeItem merge_item(const RunArgs &A, const MergeItem *items,
                                                const PassArgs &pa, int b) {
  if (!A.one_set) return items[b];
  MergeItem it;
  const int v = b / pa.items, i = b - v * pa.items;
  it.child0 = v * pa.children + i * pa.fan;
  it.nch = min(pa.fan, pa.children - i * pa.fan);
  it.off = (int64_t)v * A.n_points + (int64_t)i * pa.fan * pa.stride;
  it.stride = pa.stride;
  it.set = v;
  it.final_ = pa.items == 1;
  it.g0 = v * pa.groups;
  it.ng = pa.groups;
  it.level = pa.level;
  it.pad = 0;
  return it;
}

// One workgroup of BLK threads merges the hoods of up to BLK consecutive
// blocks of the previous level of one set (log2 BLK more rounds).  When their corners fit
// in LDS: gather them back to back, six rounds inside each wave (64
// children -> 1), then wave 0 merges the four wave hoods.  Otherwise the
// same rounds run over the workspace (global memory), each merge by a group
// of lanes, narrowing per-child intervals instead of moving corners.
// order (or null: the identity) gives the item of each launch slot, the
// largest items first.  reps > 1 (a last pass of few items): the item of slot
// i runs in workgroups i, i + items, ..., i + (reps - 1) * items.  Over the
// workspace every replica finds the
// same intervals (the rounds only read it) and gathers its own share of the
// output; otherwise replica 0 does the merge and the others stop early.
template <int BLK, int VMX>
__global__ __launch_bounds__(BLK) void merge_kernel(
    RunArgs A, const MergeItem *items, const int32_t *order, PassArgs pa,
    const int32_t *child_cnt, int32_t *cnt_out, int32_t reps) {
  // VMX corners (x, y, index) for the LDS path; the global path reuses the
  // same bytes as 1.5 * VMX corner positions (x, y)
  __shared__ __attribute__((aligned(16))) char lds_corners[VMX * 12];
  float2 *const bxy = reinterpret_cast<float2 *>(lds_corners);
  int32_t *const bid = reinterpret_cast<int32_t *>(lds_corners + VMX * 8);
  __shared__ int scum[BLK + 1];
  __shared__ int bcnt[BLK];
  __shared__ int soff[BLK];
  __shared__ int2 sblk[BLK];  // LDS path: (base, count) per child block
  __shared__ int2 sres[BLK / 2];
  __shared__ int swave[BLK / 64 + 1];
  __shared__ float4 sw4[BLK / 64];

  const int nitems = (int)gridDim.x / reps;
  const int rep = (int)blockIdx.x / nitems;        // replica of the item
  const int slot = (int)blockIdx.x - rep * nitems;  // launch slot
  const int item = order ? order[slot] : slot;
  const MergeItem it = merge_item(A, items, pa, item);
  if (rep > 0 && !it.final_) return;  // only a set's last merge is shared
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const bool fe = (A.flags & UH_FLAG_FORCE_FALLBACK) != 0;
  const bool noelim = (A.flags & UH_FLAG_NO_ELIMINATION) != 0;
  const int nch = it.nch;

  // A child is a hood, or (POINTS_FLAG) a tile's sorted surviving points.
  // Child k belongs to thread k.  Its count and its first PRE = 16 entries
  // are fetched together: load u of a wave brings entries 0..15 of four of
  // the wave's children, 16 consecutive lanes per child (entries past a
  // count are stale and ignored; indices are clamped to the workspace).
  constexpr int PRE = 16;
  const int64_t g = it.off + (int64_t)tid * it.stride;
  const uint32_t craw = tid < nch ? (uint32_t)child_cnt[it.child0 + tid] : 0u;
  // First two levels: the highest y of every child (a tile, or a group of
  // tiles) and of every group of the set outside this item are witnesses
  // (actual points of the set, earlier or later than the child).  A child
  // whose highest point beats neither the earlier nor the later witnesses
  // holds no corner and is not read.
  const bool known_max = it.level <= 1;
  float2 vx[16];
  int32_t vi[16];
  float wpre = -2.0f, wsuf = -2.0f;  // witnesses for this thread's child
  bool cand = true;
  if (known_max) {
    const float cm = tid >= nch ? -2.0f
                     : it.level == 0 ? y_decode(A.tile_max[it.child0 + tid])
                                     : y_decode(A.group_max[(it.child0 + tid) * GROUP_STRIDE]);
    // the groups this item covers: its own (level 0) or its children (level 1)
    const int glo = it.level == 0 ? item : it.child0;
    const int ghi = it.level == 0 ? item : it.child0 + nch - 1;
    float gp = -2.0f, gs = -2.0f;
    for (int k0 = 0; k0 < it.ng; k0 += 2 * BLK) {  // two loads in flight per thread
      float v[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = k0 + u * BLK + tid, gi = it.g0 + k;
        v[u] = k < it.ng && (gi < glo || gi > ghi) ? y_decode(A.group_max[gi * GROUP_STRIDE]) : -2.0f;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int gi = it.g0 + k0 + u * BLK + tid;
        if (gi < glo) gp = fmaxf(gp, v[u]);
        else gs = fmaxf(gs, v[u]);
      }
    }
    block_excl_max<BLK>(cm, gp, gs, wpre, wsuf, sw4);
    cand = noelim || cm > wpre || cm >= wsuf;
  } else {
    const int64_t last = A.n_total - 1;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int ck = (w << 6) + 4 * u + (lane >> 4);  // child of this load
      int64_t e = it.off + (int64_t)ck * it.stride + (lane & 15);
      e = e < last ? e : last;
      if (ck < nch) {
        vx[u] = A.ws_xy[e];
        vi[u] = A.ws_idx[e];
      }
    }
  }
  const bool pts = (craw & POINTS_FLAG) != 0;
  const int c = cand ? (int)(craw & ~POINTS_FLAG) : 0;
  int V;
  const int o = block_exclusive_scan<BLK>(c, swave, V);
  bcnt[tid] = c;
  soff[tid] = o;
  int npow = 1;
  while (npow < nch) npow <<= 1;
  OrientCount oc = run_counter(A);
  // the replicas share the merge over the workspace when no child is a
  // point list (chaining those rewrites the workspace in place)
  const bool shared = reps > 1 && V > VMX && !__syncthreads_or(pts);
  __syncthreads();
  if (reps > 1) {
    // The set's group maxima are zeroed for the next run once no replica
    // will read them: with witnesses (first two levels), by the last replica
    // to count itself in a counter kept in the second word of the set's
    // first group maximum (which it sets back to zero); otherwise by replica 0.
    __shared__ int s_last;
    bool zero = rep == 0;
    if (known_max) {
      uint32_t *const ticket = A.group_max + (int64_t)it.g0 * GROUP_STRIDE + 1;
      if (tid == 0) {
        s_last = atomicAdd(ticket, 1u) == (uint32_t)(reps - 1);
        if (s_last) atomicExch(ticket, 0u);
      }
      __syncthreads();
      zero = s_last != 0;
    }
    if (zero)
      for (int k = tid; k < it.ng; k += BLK) A.group_max[(it.g0 + k) * GROUP_STRIDE] = 0u;
    if (rep > 0 && !shared) return;
  }

  if (V <= VMX) {
    constexpr int NW = BLK / 64;  // waves
    bool direct = false;          // this merge is finished by the direct corner test
    int nleaf_w = 0;              // leaves of this wave's rounds
    // ---- gather: the prefetched entries to their places, then thread k
    // copies whatever child k has beyond them, eight loads in flight
    if (!known_max) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int ck = (w << 6) + 4 * u + (lane >> 4), e = lane & 15;
        if (ck < nch && e < bcnt[ck]) {
          bxy[soff[ck] + e] = vx[u];
          bid[soff[ck] + e] = vi[u];
        }
      }
    }
    // the rest: every thread copies a share of all V entries, eight loads in
    // flight, so one large child does not keep a single thread busy
    {
      const int skip = known_max ? 0 : PRE;  // entries prefetched above
      for (int e0 = 0; e0 < V; e0 += 8 * BLK) {
        float2 vx8[8];
        int32_t vi8[8];
        int dst[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * BLK + tid;
          dst[u] = -1;
          if (e < V) {
            const int k = child_of<BLK>(soff, nch, e), j = e - soff[k];
            if (j >= skip) {
              const int64_t src = it.off + (int64_t)k * it.stride + j;
              vx8[u] = A.ws_xy[src];
              vi8[u] = A.ws_idx[src];
              dst[u] = e;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (dst[u] >= 0) {
            bxy[dst[u]] = vx8[u];
            bid[dst[u]] = vi8[u];
          }
        }
      }
    }
    __syncthreads();
    // Exact elimination over the gathered corners (a sorted point list): a
    // corner is dropped when an earlier one is at least as high and a later
    // one strictly higher (the tile kernel's rule; witnesses are earlier
    // corners and later children's maxima).  Each thread filters its child
    // in place; what is left of a strictly concave chain is still one, so
    // every child stays a hood.
    {
      // A set's last merge with at most DIRECT_MAX entries gathered: the
      // direct corner test below is exact on any points in x order (removing
      // points that are no corners never changes the hood), so neither the
      // elimination nor the chains of the point lists run first.  (An earlier
      // merge filters all the same: its witnesses from the rest of the set
      // drop points its own hood would keep and pass on.)
      const bool few = !noelim && it.final_ && V <= DIRECT_MAX;
      float pre = wpre, suf = wsuf;
      if (!known_max && !few) {  // witnesses: the children's highest corners
        float cmax = -2.0f;
        for (int e0 = 0; e0 < c; e0 += 8) {  // eight LDS reads in flight
          float yv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) yv[u] = e0 + u < c ? bxy[o + e0 + u].y : -2.0f;
#pragma unroll
          for (int u = 0; u < 8; ++u) cmax = fmaxf(cmax, yv[u]);
        }
        block_excl_max<BLK>(cmax, -2.0f, -2.0f, pre, suf, sw4);
      }
      int kept = 0;
      if (noelim || few) {
        kept = c;  // every gathered corner stays
      } else if (__syncthreads_or(c > 64)) {
        // Some child is large (an arc's steep end tiles, where nearly every
        // point is a corner): the filter is shared by all threads, thread t
        // taking entries [t * Jd, t * Jd + Jd) of the V gathered ones.  (Past
        // 64 entries in one child the per-child loop below costs more:
        // arc_2^24 took 0.223 ms per step with the shared filter past 256
        // entries and 0.213 ms past 64, the mixed batch 1.860 and 1.842 ms;
        // past 16 the parabola batch slowed by 1.5 %.)  An entry
        // needs the highest earlier entry of its own child (a segmented
        // prefix maximum over the threads) and, if kept, its rank among its
        // child's kept entries (a segmented prefix sum); then the kept
        // entries move to the front of their child's segment.
        float *const fpre = reinterpret_cast<float *>(sres);  // [BLK] per child
        float *const fsuf = reinterpret_cast<float *>(scum);  // [BLK] per child
        __shared__ float fsv[BLK / 64];
        __shared__ int fsi[BLK / 64], fsh[BLK / 64];
        if (tid < nch) {
          fpre[tid] = pre;
          fsuf[tid] = suf;
        }
        bcnt[tid] = 0;  // kept per child, filled below
        __syncthreads();
        constexpr int J = (VMX + BLK - 1) / BLK;  // at most J entries per thread
        const int Jd = (V + BLK - 1) / BLK;        // this merge's: every thread takes a share
        const int e0 = tid * Jd;
        const int k0 = e0 < V ? child_of<BLK>(soff, nch, e0) : 0;
        // Each walk over the thread's entries keeps its child's bounds and
        // witnesses in registers and reads them from LDS only where it passes
        // into the next child: the entries' own reads do not wait on a walk.
        const int cs0 = soff[k0];                         // first entry of child k0
        const int ce0 = k0 + 1 < nch ? soff[k0 + 1] : V;  // ... and past its last
        const bool starts = e0 < V && cs0 == e0;  // the chunk starts a child
        // child k holds [cs, ce): move on to the child holding e
        auto step = [&](int e, int &k, int &cs, int &ce) {
          while (e >= ce) {
            ++k;
            cs = ce;
            ce = k + 1 < nch ? soff[k + 1] : V;
          }
        };
        bool head = false;
        float m = -INFINITY;
        {
          int k = k0, cs = cs0, ce = ce0;
          for (int j = 0; j < Jd && e0 + j < V; ++j) {
            const int e = e0 + j;
            const float y = bxy[e].y;
            step(e, k, cs, ce);
            if (cs == e) {
              head = true;
              m = y;
            } else {
              m = fmaxf(m, y);
            }
          }
        }
        const float mcarry = seg_excl_scan<BLK, float>(
            head, m, -INFINITY, [](float a, float b) { return fmaxf(a, b); }, fsv, fsh);
        uint32_t keepbits = 0;
        int nkept = 0;
        bool khead = false;
        {
          int k = k0, cs = cs0, ce = ce0;
          float fp = fpre[k0], fs = fsuf[k0];
          float run = starts ? -INFINITY : mcarry;
          for (int j = 0; j < Jd && e0 + j < V; ++j) {
            const int e = e0 + j;
            const float y = bxy[e].y;
            if (e >= ce) {
              step(e, k, cs, ce);
              fp = fpre[k];
              fs = fsuf[k];
            }
            if (cs == e) {
              run = -INFINITY;
              khead = true;
              nkept = 0;
            }
            if (y > fmaxf(fp, run) || y >= fs) {
              keepbits |= 1u << j;
              ++nkept;
            }
            run = fmaxf(run, y);
          }
        }
        const int rcarry = seg_excl_scan<BLK, int>(
            khead, nkept, 0, [](int a, int b) { return a + b; }, fsi, fsh);
        float2 qv[J];
        int32_t iv[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
          if (j < Jd && e0 + j < V) {
            qv[j] = bxy[e0 + j];
            iv[j] = bid[e0 + j];
          }
        }
        __syncthreads();  // every entry is read before any moves
        {
          int k = k0, cs = cs0, ce = ce0;
          int r = starts ? 0 : rcarry;
#pragma unroll
          for (int j = 0; j < J; ++j) {
            const int e = e0 + j;
            if (j < Jd && e < V) {
              step(e, k, cs, ce);
              if (cs == e) r = 0;
              if ((keepbits >> j) & 1u) {
                bxy[cs + r] = qv[j];
                bid[cs + r] = iv[j];
                ++r;
              }
              // the thread holding a child's last entry knows its count: one
              // plain store per child, no atomic per kept entry
              if (e + 1 == ce) bcnt[k] = r;
            }
          }
        }
        __syncthreads();
        kept = tid < nch ? bcnt[tid] : 0;
      } else {
        // each thread filters its own child in place
        for (int e0 = 0; e0 < c; e0 += 8) {  // a batch is read before it is rewritten
          float2 qv[8];
          int32_t iv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (e0 + u < c) {
              qv[u] = bxy[o + e0 + u];
              iv[u] = bid[o + e0 + u];
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (e0 + u < c) {
              const bool keep = qv[u].y > pre || qv[u].y >= suf;
              pre = fmaxf(pre, qv[u].y);
              if (keep) {
                bxy[o + kept] = qv[u];
                bid[o + kept] = iv[u];
                ++kept;
              }
            }
          }
        }
      }
      // Few entries left: the workgroup finishes the merge by testing every
      // entry against the hood's definition directly, whose depth beats that
      // of log2(leaves) rounds of merges; the test takes any points, so the
      // point lists need no hoods first.  Otherwise a point-list child
      // becomes a hood (the serial strip hood of its surviving points, the
      // paper's serial hoods of small strips), the leaves are dealt to the
      // waves in contiguous runs of at most `per`, each wave runs the rounds
      // over its run, and the wave hoods are joined pairwise in log2(waves)
      // rounds.
      int vk = kept;
      for (int d = 1; d < 64; d <<= 1) vk += __shfl_xor(vk, d, 64);
      if (lane == 0) sres[w] = make_int2(vk, 0);
      __syncthreads();
      int vsum = 0;
      for (int k = 0; k < NW; ++k) vsum += sres[k].x;
      direct = !noelim && vsum <= DIRECT_MAX;
      if (pts && kept > 0 && !direct) kept = chain_inplace(bxy + o, bid + o, kept, oc, fe);
      // leaves: the non-empty children, in order
      const uint64_t ne = __ballot(kept > 0);
      if (lane == 0) swave[w] = __builtin_popcountll(ne);
      __syncthreads();
      int before = 0, total = 0;
      for (int k = 0; k < NW; ++k) {
        before += k < w ? swave[k] : 0;
        total += swave[k];
      }
      const int per = total > 0 ? (total + NW - 1) / NW : 1;
      if (kept > 0) {
        const int li = before + __builtin_popcountll(ne & ((1ull << lane) - 1ull));
        const int wv = li / per;
        sblk[direct ? li : (wv << 6) + li - wv * per] = make_int2(o, kept);
      }
      if (tid == 0) swave[NW] = total;
      nleaf_w = min(max(total - w * per, 0), per);
    }
    __syncthreads();
    if (direct) {
      // the partial results between the first 64 corner slots and the indices
      static_assert(1024 + NW * 64 * 20 <= VMX * 8, "direct test scratch overlaps the indices");
      block_direct_hood<NW>(bxy, bid, sblk, swave[NW], oc, fe,
                            reinterpret_cast<float4 *>(lds_corners + 1024),
                            reinterpret_cast<int *>(lds_corners + 1024 + NW * 64 * 16));
      __syncthreads();
    } else {
      if (nleaf_w > 0) {
        const int2 lf = lane < nleaf_w ? sblk[(w << 6) + lane] : make_int2(0, 0);
        const int2 hood = wave_rounds(bxy, bid, lf, nleaf_w, oc, fe);
        if (lane == 0) sblk[w << 6] = hood;
      } else if (lane == 0) {
        sblk[w << 6] = make_int2(0, 0);
      }
      __syncthreads();
      for (int st = 1; st < NW; st <<= 1) {  // join the wave hoods pairwise
        if ((w & (2 * st - 1)) == 0 && w + st < NW) {
          const int2 P = sblk[w << 6], Q = sblk[(w + st) << 6];
          int nb, nc;
          merge_blocks(bxy, bid, P.x, P.y, Q.x, Q.y, 6, lane, 0, nb, nc, oc, fe);
          wave_sync();
          if (lane == 0) sblk[w << 6] = make_int2(nb, nc);
        }
        __syncthreads();
      }
    }
    if (w == 0) {
      const int hb = sblk[0].x, hc = sblk[0].y;
      if (it.final_) {
        int32_t *dst = A.out_idx + set_base(A, it.set);
        for (int k = lane; k < hc; k += 64) dst[k] = bid[hb + k];
        if (lane == 0) {
          const int st = A.set_status[it.set];
          A.out_counts[it.set] = st ? st : hc;
          if (st) A.set_status[it.set] = 0;  // zero again for the next run
          finish_stats(A, it.set, st);
        }
      } else {
        for (int k = lane; k < hc; k += 64) {
          A.ws_xy[it.off + k] = bxy[hb + k];
          A.ws_idx[it.off + k] = bid[hb + k];
        }
        if (lane == 0) cnt_out[item] = hc;
      }
    }
    if (it.final_ && reps == 1)  // the set's group maxima, zero again for the next run
      for (int k = tid; k < it.ng; k += BLK) A.group_max[(it.g0 + k) * GROUP_STRIDE] = 0u;
    flush_wave_stats(A, it.set, oc);
    return;
  }

  // ---- too large for LDS: the same rounds over the workspace, moving no
  // corner.  A merge keeps a prefix of P and a suffix of Q, so every block
  // is a run of children, each keeping one interval [klo, klo + bcnt) of its
  // corners; a round only narrows intervals, the searches read the corners
  // where they are (Rope), and the result is gathered once at the end.
  if (pts && c > 0)  // point-list children first become hoods, in place
    bcnt[tid] = chain_inplace(A.ws_xy + g, A.ws_idx + g, c, oc, fe);
  int *const cum = scum;                           // [BLK + 1] prefix of the kept counts
  int *const klo = reinterpret_cast<int *>(sblk);  // [BLK] start of each child's kept interval
  klo[tid] = 0;
  // If the corners' positions fit in LDS (1.5 * VMX of them), copy them
  // there: child k's at soff[k] (its count before chaining is an upper bound)
  const bool in_lds = V <= VMX + VMX / 2;
  float2 *const lxy = reinterpret_cast<float2 *>(lds_corners);
  if (in_lds) {
    __syncthreads();  // the chained counts
    // a thread's positions only grow: its child, that child's slot minus its
    // first position, its count and the next child's first position stay
    // in registers and change when a position passes into the next child
    int kw = 0, kend = nch > 1 ? soff[1] : INT32_MAX, kcnt = bcnt[0];
    int64_t kbase = it.off;
    auto child_at = [&](int e) {  // moves the cached child forward to e's
      if (e >= kend) {
        do ++kw;
        while (kw + 1 < nch && soff[kw + 1] <= e);
        kbase = it.off + (int64_t)kw * it.stride - soff[kw];
        kend = kw + 1 < nch ? soff[kw + 1] : INT32_MAX;
        kcnt = bcnt[kw] + soff[kw];
      }
    };
    // four consecutive positions per thread step: one wide load where the
    // four are kept corners of one child (positions past a child's kept
    // corners are skipped), eight such steps in flight
    for (int e0 = 0; e0 < V; e0 += 4 * 8 * BLK) {
      Xy4 v8[8];
      uint32_t wide = 0u, some = 0u;  // step u is one wide load / position 4u + q is kept
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 4 * (u * BLK + tid);
        if (e < V) {
          child_at(e);
          if (e + 3 < kcnt) {  // kcnt <= kend: all four in this child, all kept
            __builtin_memcpy(&v8[u], A.ws_xy + kbase + e, sizeof(Xy4));
            wide |= 1u << u;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              v8[u].v[q] = make_float2(0.f, 0.f);
              if (e + q < V) {
                child_at(e + q);
                if (e + q < kcnt) {
                  v8[u].v[q] = A.ws_xy[kbase + e + q];
                  some |= 1u << (4 * u + q);
                }
              }
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 4 * (u * BLK + tid);
        if ((wide >> u) & 1u) {
#pragma unroll
          for (int q = 0; q < 4; ++q) lxy[e + q] = v8[u].v[q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if ((some >> (4 * u + q)) & 1u) lxy[e + q] = v8[u].v[q];
        }
      }
    }
  }
  auto rescan = [&]() {
    __syncthreads();
    int tot;
    cum[tid] = block_exclusive_scan<BLK>(tid < nch ? bcnt[tid] : 0, swave, tot);
    if (tid == 0) cum[BLK] = tot;
    __syncthreads();
  };
  rescan();
#pragma unroll 1
  for (int j = 0; (1 << j) < nch; ++j) {
    const int M = npow >> (j + 1);
    const int G = BLK / M;
    const int m = tid / G, t = tid % G;
    const int lp = (2 * m) << j, lq = (2 * m + 1) << j;
    const int le = min((2 * m + 2) << j, nch);
    const bool active = lq < nch;
    int a = -1, b = 0;
    if (active) {
      Rope P{A.ws_xy, cum, klo, it.off, it.stride, lp, lq, cum[lp]};
      Rope Q{A.ws_xy, cum, klo, it.off, it.stride, lq, le, cum[lq]};
      if (in_lds) {
        P.lxy = Q.lxy = lxy;
        P.lbase = Q.lbase = soff;
      }
      P.prep();
      Q.prep();
      int hp = cum[lq] - cum[lp], qs = 0;
      const int hq = cum[le] - cum[lq];
      if (hp > 0 && hq > 0) junction_rule(P[hp - 1], Q[0], hp, qs);
      const int hqe = hq - qs;
      a = hp - 1;
      Q.c0 += qs;
      const int L = G < 64 ? G : 64;
      if (hp > 0 && hqe > 0 && t < L)
        bridge_find<Rope>(P, hp, Q, hqe, L, t, (tid & 63) - t, a, b, oc, fe);
      b += qs;  // Q's first kept corner
    }
    __syncthreads();  // searches done; every merge's result to sres
    if (t == 0) sres[m] = active ? make_int2(a + 1, b) : make_int2(INT32_MAX, 0);
    __syncthreads();
    if (tid < nch) {  // child tid narrows its interval
      const int mk = tid >> (j + 1);
      const int2 r = sres[mk];
      const int lpk = (2 * mk) << j, lqk = (2 * mk + 1) << j;
      const int cnt = bcnt[tid];
      if (tid < lqk) {  // in P: keeps P's corners below r.x
        bcnt[tid] = min(max(r.x - (cum[tid] - cum[lpk]), 0), cnt);
      } else {  // in Q: drops Q's corners below r.y
        const int drop = min(max(r.y - (cum[tid] - cum[lqk]), 0), cnt);
        klo[tid] += drop;
        bcnt[tid] = cnt - drop;
      }
    }
    rescan();
  }
  // the result: corner e lives in child l with cum[l] <= e < cum[l + 1].  A
  // thread's positions only grow, so its child is found by walking forward
  // from the previous one (each child passed once) instead of a search.
  // Replica r gathers corners [e_lo, e_hi) of a set's last merge.
  const int hc = cum[BLK];
  const int share = it.final_ ? (((hc + reps - 1) / reps + 3) & ~3) : hc;
  const int e_lo = min(rep * share, hc), e_hi = min(e_lo + share, hc);
  int lw = child_of<BLK>(cum, nch, e_lo);         // the child of the last position,
  int64_t lbase = it.off + (int64_t)lw * it.stride + klo[lw] - cum[lw];  // its position minus its first rank,
  int lend = lw + 1 < nch ? cum[lw + 1] : INT32_MAX;  // and the rank where the next one starts
  auto where = [&](int e) {
    if (e >= lend) {
      do ++lw;
      while (lw + 1 < nch && cum[lw + 1] <= e);
      lbase = it.off + (int64_t)lw * it.stride + klo[lw] - cum[lw];
      lend = lw + 1 < nch ? cum[lw + 1] : INT32_MAX;
    }
    return lbase + e;
  };
  if (it.final_) {
    int32_t *dst = A.out_idx + set_base(A, it.set);
    // four consecutive corners per thread step (one wide load where they
    // lie in one child), eight steps in flight
    for (int e0 = e_lo; e0 < e_hi; e0 += 4 * 8 * BLK) {
      Idx4 vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 4 * (u * BLK + tid);
        if (e < e_hi) {
          const int64_t p = where(e);
          if (e + 3 < lend && e + 3 < e_hi) {
            __builtin_memcpy(&vi[u], A.ws_idx + p, sizeof(Idx4));
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              vi[u].v[q] = e + q < e_hi ? A.ws_idx[where(e + q)] : 0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 4 * (u * BLK + tid);
        if (e + 3 < e_hi) {
          __builtin_memcpy(dst + e, &vi[u], sizeof(Idx4));
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (e + q < e_hi) dst[e + q] = vi[u].v[q];
        }
      }
    }
    if (tid == 0 && rep == 0) {
      const int st = A.set_status[it.set];
      A.out_counts[it.set] = st ? st : hc;
      if (st) A.set_status[it.set] = 0;  // zero again for the next run
      finish_stats(A, it.set, st);
    }
  } else {
    // compact to the item's slot: corner e comes from at or after slot
    // position e (a child keeps at most its slot's length), so a chunk read
    // whole before it is written never overwrites a corner still to be read;
    // the next chunk reads only at or after its own first position, past
    // every position this one writes, so it needs no wait for these writes.
    // Four consecutive corners per thread step, eight steps in flight.
    for (int e0 = 0; e0 < hc; e0 += 4 * 8 * BLK) {
      Xy4 vx[8];
      Idx4 vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 4 * (u * BLK + tid);
        if (e < hc) {
          const int64_t p = where(e);
          if (e + 3 < lend && e + 3 < hc) {
            __builtin_memcpy(&vx[u], A.ws_xy + p, sizeof(Xy4));
            __builtin_memcpy(&vi[u], A.ws_idx + p, sizeof(Idx4));
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              vx[u].v[q] = make_float2(0.f, 0.f);
              vi[u].v[q] = 0;
              if (e + q < hc) {
                const int64_t pq = where(e + q);
                vx[u].v[q] = A.ws_xy[pq];
                vi[u].v[q] = A.ws_idx[pq];
              }
            }
          }
        }
      }
      __syncthreads();  // the chunk is read whole before any of it is written
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 4 * (u * BLK + tid);
        if (e + 3 < hc) {
          __builtin_memcpy(A.ws_xy + it.off + e, &vx[u], sizeof(Xy4));
          __builtin_memcpy(A.ws_idx + it.off + e, &vi[u], sizeof(Idx4));
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (e + q < hc) {
              A.ws_xy[it.off + e + q] = vx[u].v[q];
              A.ws_idx[it.off + e + q] = vi[u].v[q];
            }
          }
        }
      }
    }
    if (tid == 0) cnt_out[item] = hc;
  }
  if (it.final_ && reps == 1)  // the set's group maxima, zero again for the next run
    for (int k = tid; k < it.ng; k += BLK) A.group_max[(it.g0 + k) * GROUP_STRIDE] = 0u;
  if (rep == 0) flush_wave_stats(A, it.set, oc);
}

// ------------------------------------------------------------ convex hull
// Joins the two hoods of one set into its convex hull, counter-clockwise:
// the lower hood left to right, then the upper hood right to left without
// the corners the two share at either end.  hood: upper hood at [0, n),
// lower at [n, 2n); cnt: their counts (or the set's data-error status).
__global__ void hull_assemble_kernel(const int32_t *hood, const int32_t *cnt, int64_t n,
                                     int32_t *out_idx, int32_t *out_count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cnt[0] <= 0 || cnt[1] <= 0) {  // an empty set, or a data error (reported by both hoods)
    if (t == 0) *out_count = min(cnt[0], cnt[1]);
    return;
  }
  // a hood never has more than n corners, nor the hull (every index at most
  // once); the clamps only keep the accesses inside the buffers
  const int32_t hu = (int32_t)min((int64_t)cnt[0], n), hl = (int32_t)min((int64_t)cnt[1], n);
  const int32_t *up = hood, *lo = hood + n;
  const bool skip_right = up[hu - 1] == lo[hl - 1];
  const int32_t k_hi = hu - 1 - (skip_right ? 1 : 0);  // upper corners kept: k_hi down to k_lo
  const int32_t k_lo = up[0] == lo[0] ? 1 : 0;
  const int32_t nup = k_hi >= k_lo ? k_hi - k_lo + 1 : 0;
  const int64_t total = min((int64_t)hl + nup, n);
  for (int64_t e = t; e < total; e += (int64_t)gridDim.x * blockDim.x)
    out_idx[e] = e < hl ? lo[e] : up[k_hi - (e - hl)];
  if (t == 0) *out_count = (int32_t)total;
}

// --------------------------------------------------------- unsorted input
// Maps the corners of every (virtual) set from sorted positions back to
// set-relative input indices: out[k] = perm[set start + out[k]].  One
// workgroup per set; the set of a lower hood is set - in_sets.
__global__ void unsort_kernel(const int64_t *set_start, int32_t in_sets, const int32_t *perm,
                              int32_t *out_idx, const int32_t *out_counts) {
  const int v = blockIdx.x;
  const int32_t c = out_counts[v];
  const int64_t src = set_start[v < in_sets ? v : v - in_sets];
  const int64_t n = set_start[(v < in_sets ? v : v - in_sets) + 1] - src;
  int32_t *o = out_idx + set_start[v];
  for (int k = threadIdx.x; k < c; k += blockDim.x) {
    const int32_t q = o[k];
    if (q >= 0 && q < n) o[k] = perm[src + q];  // always, for a hood of the set
  }
}

// Debug trace of one level of the merge tree (the paper's per-stage dump of
// every block's hood): block b of `level` (0: the tiles, k: the items of
// merge pass k) writes its corners' set-relative indices at out_idx + its
// first point and its count (bit 31: a tile's sorted surviving points rather
// than a hood) to out_counts[b].  A block that finished its set wrote both to
// the run's outputs already (A.out_idx, A.out_counts), where they are read.
__global__ void trace_kernel(RunArgs A, int32_t level, int32_t tiles_per_set,
                             const TileItem *tiles, const MergeItem *items, PassArgs pa,
                             const int32_t *cnt, int32_t *out_counts) {
  const int b = blockIdx.x;
  int64_t start;
  int set;
  bool fin;
  if (level == 0) {
    if (A.one_set) {
      const int v = b / tiles_per_set, t = b - v * tiles_per_set;
      start = (int64_t)v * A.n_points + (int64_t)t * A.tile_len;
      set = v;
      fin = tiles_per_set == 1;
    } else {
      const TileItem it = tiles[b];
      start = it.start;
      set = it.set;
      fin = it.rel0 == 0 && it.len == it.set_len;
    }
  } else {
    const MergeItem it = merge_item(A, items, pa, b);
    start = it.off;
    set = it.set;
    fin = it.final_ != 0;
  }
  const int32_t c = fin ? A.out_counts[set] : cnt[b];
  if (!fin) {
    const int32_t m = (int32_t)((uint32_t)c & ~POINTS_FLAG);
    for (int k = threadIdx.x; k < m; k += blockDim.x) A.out_idx[start + k] = A.ws_idx[start + k];
  }
  if (threadIdx.x == 0) out_counts[b] = c;
}

// Writes `value` to out[0 .. m) (counts of empty single-set runs).
__global__ void fill_kernel(int32_t *out, int32_t m, int32_t value) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) out[t] = value;
}

// ---------------------------------------------------------------- probes
__global__ void bridge_kernel(const float2 *P, int hp, const float2 *Q, int hq,
                              int L, int32_t *out_ab) {
  const int t = threadIdx.x;
  OrientCount oc;
  int a = -1, b = -1;
  if (t < L) bridge_search<const float2 *>(P, hp, Q, hq, L, t, 0, a, b, oc, false);
  if (t == 0) {
    out_ab[0] = a;
    out_ab[1] = b;
  }
}

__global__ void orient_kernel(const float2 *a, const float2 *b, const float2 *c,
                              int64_t m, int8_t *out, uint8_t *fb, int force) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  OrientCount oc;
  out[i] = (int8_t)orient_sign(a[i], b[i], c[i], oc, force != 0);
  if (fb) fb[i] = (uint8_t)(oc.fallbacks != 0);
}

}  // namespace uh

// ====================================================================== host
using namespace uh;

struct upper_hull_plan;

namespace {

constexpr int MAX_PASSES = 40;

// Merge passes of a single set of n points (with both hoods, two mirrored
// sets of n points): the shape of every pass follows from n, K and F.
struct SingleShape {
  int64_t n = 0;
  bool both = false;
  int K = 16, T = 1024, F = 256;
  int32_t VS = 1;         // sets: 1, or 2 with both hoods
  int32_t tiles = 0;      // per set
  int32_t groups = 0;     // first-level merge items per set
  int32_t group_fan = 1;  // tiles per first-level item
  int npass = 0;
  PassArgs pass[MAX_PASSES];
  bool wide[MAX_PASSES];
};

// Everything one run enqueues.
struct Launch {
  RunArgs A;
  int32_t S = 0;             // sets (with both hoods: both halves)
  int32_t tile_grid = 0;     // tile kernel workgroups (with both hoods: the upper half)
  int K = 16;
  bool both = false;
  const TileItem *tiles = nullptr;
  int32_t *cnt0 = nullptr;
  int npass = 0;
  int32_t pass_items[MAX_PASSES];
  int32_t pass_reps[MAX_PASSES];  // workgroups per item (merge_kernel's reps)
  bool pass_wide[MAX_PASSES];
  const MergeItem *items[MAX_PASSES];
  const int32_t *order[MAX_PASSES];  // launch slot -> item (null: identity)
  int32_t *cnt[MAX_PASSES];
  PassArgs pa[MAX_PASSES];
  bool init = false;         // launch init_kernel first
  int32_t init_groups = 0;   // group maxima it clears
  hipEvent_t probe_before = nullptr, probe_after = nullptr;
};

int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus;
}

// Default fan-in: 256, the fewest merge passes, for every plan.  A "large"
// plan (at least 8 tiles per compute unit) is flagged for the choice of the
// wide merge workgroup.  (Halving the fan-in until the first merge pass has
// an item per compute unit was slower, once the merges had become short:
// arc_2^24 took 0.2593 ms per step at fan-in 64 and 0.2438 ms at 256,
// uniform_2^27 0.2665 ms at 64, 0.2479 ms at 128 and 0.2289 ms at 256; the
// mixed batch 1.97, 1.90 and 1.86 ms.  A pass fewer saves more than the
// idle units of a first pass of few items cost.)
int default_fan_in(const int64_t *off, int32_t S, int T, int cus, bool *large) {
  int64_t all_tiles = 0;
  for (int32_t s = 0; s < S; ++s) all_tiles += (off[s + 1] - off[s] + T - 1) / T;
  *large = all_tiles >= 8 * (int64_t)cus;
  return BLOCK;
}

// Workgroups per item of the last merge pass (all of its items are final
// merges).  A last pass of few items runs each in several workgroups, which
// share the gathering of a large hood: one workgroup gathers some 11 bytes
// per cycle, about 23 us for the 45 800 corners of arc_2^24's hood.
int32_t last_pass_reps(int32_t items, int cus) {
  if (items <= 0 || items > 8) return 1;
  return std::max(1, std::min(32, cus / (8 * items)));
}

// The passes of a single-set run, by the rules of upper_hull_plan_create.
void single_shape(int64_t n, bool both, int K, int F, bool large, SingleShape &sh) {
  sh.n = n;
  sh.both = both;
  sh.K = K;
  sh.T = 64 * K;
  sh.F = F;
  sh.VS = both ? 2 : 1;
  sh.tiles = (int32_t)((n + sh.T - 1) / sh.T);
  sh.npass = 0;
  sh.groups = 0;
  sh.group_fan = F;
  int64_t stride = sh.T;
  int32_t count = sh.tiles;
  while (count > 1 && sh.npass < MAX_PASSES) {
    // a set with BLOCK + 1 .. WIDE blocks left finishes in one wide workgroup
    const bool use_wide = F == BLOCK && count > BLOCK && count <= WIDE;
    const int32_t FS = use_wide ? WIDE : F;
    const int32_t items = (count + FS - 1) / FS;
    PassArgs &pa = sh.pass[sh.npass];
    pa.stride = stride;
    pa.children = count;
    pa.fan = FS;
    pa.items = items;
    pa.level = std::min(sh.npass, 2);
    pa.pad = 0;
    // the wide workgroup for more than BLOCK children, and in a large plan
    // for a pass of few items, whose merges are large and latency-bound
    sh.wide[sh.npass] = (large && (int64_t)items * sh.VS <= 64) || FS > BLOCK;
    if (sh.npass == 0) {
      sh.groups = items;
      sh.group_fan = FS;
    }
    ++sh.npass;
    count = items;
    stride *= F;
  }
  for (int k = 0; k < sh.npass; ++k) sh.pass[k].groups = sh.groups;
}

// Byte layout of a single-set run's working memory (256-byte aligned parts).
struct SingleLayout {
  size_t status = 0, group_max = 0, tile_max = 0, cnt0 = 0, ws_idx = 0, ws_xy = 0;
  size_t hull_idx = 0, hull_cnt = 0, total = 0;
  size_t cnt[MAX_PASSES];
};

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace bytes that serve every single-set or batched-free call with at
// most m points over at most s sets: tiles of T = 1024 points (each set adds
// at most one partial tile); first-level items of at least 64 tiles (or one
// per set); items of all later passes together at most the tiles; the parts'
// 256-byte alignment; and, for two sets or more, the hood buffers of
// convex_hull (4 bytes per point).
constexpr size_t workspace_bound(size_t m, size_t s) {
  const size_t tiles = (m + 1023) / 1024 + s;
  const size_t groups = tiles / 64 + 1 + s;
  size_t b = 0;
  b += align256(4 * s);                          // status
  b += align256(4 * GROUP_STRIDE * groups);      // group maxima
  b += 2 * align256(4 * tiles);                  // tile maxima, tile counts
  b += align256(4 * tiles) + MAX_PASSES * 256;   // pass counts
  b += align256(4 * m) + align256(8 * m);        // corner indices and positions
  if (s >= 2) b += align256(4 * m) + align256(4 * s);  // hood buffers
  return b;
}

SingleLayout single_layout(const SingleShape &sh, bool hull_buffers) {
  SingleLayout L;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t here = at;
    at += align256(std::max<size_t>(bytes, 4));
    return here;
  };
  const size_t VS = (size_t)sh.VS, N = VS * (size_t)sh.n;
  L.status = take(4 * VS);
  L.group_max = take(4 * GROUP_STRIDE * VS * (size_t)sh.groups);
  L.tile_max = take(4 * VS * (size_t)sh.tiles);
  L.cnt0 = take(4 * VS * (size_t)sh.tiles);
  for (int k = 0; k < sh.npass; ++k) L.cnt[k] = take(4 * VS * (size_t)sh.pass[k].items);
  L.ws_idx = take(4 * N);
  L.ws_xy = take(8 * N);
  if (hull_buffers) {
    L.hull_idx = take(4 * N);
    L.hull_cnt = take(4 * VS);
  }
  L.total = at;
  return L;
}

template <class T>
int dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, count * sizeof(T)) == hipSuccess ? UH_OK : UH_ERR_ALLOC;
}

template <class T>
int upload(T *dst, const std::vector<T> &src) {
  if (src.empty()) return UH_OK;
  return hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) ==
                 hipSuccess
             ? UH_OK
             : UH_ERR_HIP;
}

int capturing(hipStream_t stream, bool *yes) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return UH_ERR_HIP;
  *yes = cs != hipStreamCaptureStatusNone;
  return UH_OK;
}

int enqueue(const Launch &L, hipStream_t stream) {
  const RunArgs &A = L.A;
  if (L.init) {
    const int m = std::max(L.S, L.init_groups);
    hipLaunchKernelGGL(init_kernel, dim3((m + 255) / 256), dim3(256), 0, stream, L.S,
                       L.init_groups, A);
  }
  if (L.tile_grid > 0) {
    const dim3 blk(64);
    if (L.probe_before && hipEventRecord(L.probe_before, stream) != hipSuccess) return UH_ERR_HIP;
#define UH_TILE(KK, BB)                                                                     \
  hipLaunchKernelGGL((tile_kernel<KK, BB>), dim3(L.tile_grid), blk, 0, stream, A, L.tiles, \
                     L.cnt0, L.tile_grid)
    switch (L.K * 2 + (L.both ? 1 : 0)) {
      case 8: UH_TILE(4, false); break;
      case 9: UH_TILE(4, true); break;
      case 16: UH_TILE(8, false); break;
      case 17: UH_TILE(8, true); break;
      case 32: UH_TILE(16, false); break;
      case 33: UH_TILE(16, true); break;
      case 64: UH_TILE(32, false); break;
      case 65: UH_TILE(32, true); break;
      default: return UH_ERR_ARG;
    }
#undef UH_TILE
    if (L.probe_after && hipEventRecord(L.probe_after, stream) != hipSuccess) return UH_ERR_HIP;
  }
  for (int ps = 0; ps < L.npass; ++ps) {
    const int32_t *ccnt = ps == 0 ? L.cnt0 : L.cnt[ps - 1];
    const int32_t reps = L.pass_reps[ps];
    const dim3 grid((unsigned)(L.pass_items[ps] * reps));
    if (L.pass_wide[ps])
      hipLaunchKernelGGL((merge_kernel<WIDE, VMAX_WIDE>), grid, dim3(WIDE), 0, stream, A,
                         L.items[ps], L.order[ps], L.pa[ps], ccnt, L.cnt[ps], reps);
    else
      hipLaunchKernelGGL((merge_kernel<BLOCK, VMAX>), grid, dim3(BLOCK), 0, stream, A,
                         L.items[ps], L.order[ps], L.pa[ps], ccnt, L.cnt[ps], reps);
  }
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

}  // namespace

struct upper_hull_plan {
  int device = 0;
  int32_t S = 0;
  int64_t N = 0;
  int K = 16, T = 4096, F = 256;
  uint32_t flags = 0;
  bool both = false;       // upper and lower hood: S, N, ntiles, ngroups count both
  int32_t in_S = 0;        // input sets
  int64_t in_N = 0;        // input points
  int32_t ntiles = 0;
  bool has_empty = false;  // some set has no points
  int32_t ngroups = 0;     // first-level merge items
  int32_t group_fan = 1;   // single set: tiles per first-level item
  SingleShape single;      // a plan of one input set: its passes follow from n
  std::vector<int64_t> h_voff;               // set starts (both halves)
  std::vector<TileItem> h_tiles;             // host copies of the tables (more
  std::vector<std::vector<MergeItem>> h_items;  // than one set), for the trace
  int32_t *trace_cnt = nullptr;              // run counts of upper_hull_plan_trace
  uint32_t *tile_max = nullptr, *group_max = nullptr;
  std::vector<int32_t> pass_items;  // merge items per pass
  int32_t last_reps = 1;            // workgroups per item of the last pass
  std::vector<char> pass_wide;      // per pass: the wide merge workgroup
  // device memory
  int64_t *d_set_start = nullptr;
  TileItem *d_tiles = nullptr;
  int32_t *d_cnt0 = nullptr;
  std::vector<MergeItem *> d_items;
  std::vector<int32_t *> d_order;  // per pass: launch slot -> item (null: identity)
  std::vector<int32_t *> d_cnt;   // per pass: item corner counts
  float2 *ws_xy = nullptr;
  int32_t *ws_idx = nullptr;
  int32_t *set_status = nullptr;
  // graph cache: (points, out_idx, out_counts, stats) -> exec, least recently
  // used first; at most GRAPH_CACHE entries
  static constexpr size_t GRAPH_CACHE = 8;
  std::vector<std::pair<std::tuple<const void *, void *, void *, void *>, hipGraphExec_t>> graphs;
  hipStream_t cap_stream = nullptr;
  hipEvent_t probe_before = nullptr, probe_after = nullptr;
  bool unsorted = false;            // sort every set by x first (UH_FLAG_UNSORTED)
  uh_rs::RadixPlan rs;
  float2 *sorted = nullptr;         // [in_N] the points in sorted order
  int32_t *perm = nullptr;          // [in_N] their set-relative input indices
  std::mutex mu;
};

namespace {

void free_plan_memory(upper_hull_plan *p) {
  (void)hipFree(p->d_set_start);
  (void)hipFree(p->d_tiles);
  (void)hipFree(p->d_cnt0);
  for (auto *q : p->d_items) (void)hipFree(q);
  for (auto *q : p->d_order) (void)hipFree(q);
  for (auto *q : p->d_cnt) (void)hipFree(q);
  (void)hipFree(p->ws_xy);
  (void)hipFree(p->ws_idx);
  (void)hipFree(p->set_status);
  (void)hipFree(p->tile_max);
  (void)hipFree(p->group_max);
  uh_rs::radix_plan_free(&p->rs);
  (void)hipFree(p->sorted);
  (void)hipFree(p->perm);
  (void)hipFree(p->trace_cnt);
  for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
}

Launch plan_launch(upper_hull_plan *p, const RunArgs &A, bool with_stats) {
  Launch L;
  L.A = A;
  L.S = p->S;
  L.tile_grid = p->both ? p->ntiles / 2 : p->ntiles;  // one wave per input tile does both hoods
  L.K = p->K;
  L.both = p->both;
  L.tiles = p->d_tiles;
  L.cnt0 = p->d_cnt0;
  L.npass = (int)p->pass_items.size();
  for (int k = 0; k < L.npass; ++k) {
    L.pass_items[k] = p->pass_items[k];
    L.pass_reps[k] = k + 1 == L.npass ? p->last_reps : 1;
    L.pass_wide[k] = p->pass_wide[k] != 0;
    L.items[k] = p->d_items.empty() ? nullptr : p->d_items[k];
    L.order[k] = p->d_order.empty() ? nullptr : p->d_order[k];
    L.cnt[k] = p->d_cnt[k];
    L.pa[k] = p->in_S == 1 ? p->single.pass[k] : PassArgs{};
  }
  // Per-set status starts at zero (plan creation) and the final merge of a
  // set that saw an error zeroes it again, so the clearing pass is needed
  // only for stats counters and for empty sets' counts.
  L.init = with_stats || p->has_empty;
  L.init_groups = 0;
  L.probe_before = p->probe_before;
  L.probe_after = p->probe_after;
  return L;
}

int enqueue_run(upper_hull_plan *p, const RunArgs &A0, hipStream_t stream) {
  RunArgs A = A0;
  if (p->unsorted) {  // the sort by x in front: the hull reads the sorted copy
    const int rc = uh_rs::radix_sort_enqueue(p->rs, A0.pts, p->in_N, p->sorted, p->perm, stream);
    if (rc) return rc;
    A.pts = p->sorted;
  }
  int rc = enqueue(plan_launch(p, A, A.stats != nullptr), stream);
  if (rc) return rc;
  if (p->unsorted)
    hipLaunchKernelGGL(unsort_kernel, dim3(p->S), dim3(256), 0, stream, p->d_set_start, p->in_S,
                       p->perm, A.out_idx, A.out_counts);
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

// ---- workspaces of the single-set calls
struct Workspace {
  void *ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<int, Workspace> g_user_ws;                           // device -> caller's workspace
std::map<std::pair<int, hipStream_t>, Workspace> g_lib_ws;    // (device, stream) -> library's

// The workspace a single-set call on `stream` uses, at least `need` bytes.
int single_workspace(size_t need, hipStream_t stream, void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UH_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_ws_mu);
  auto u = g_user_ws.find(dev);
  if (u != g_user_ws.end()) {
    if (u->second.bytes < need) return UH_ERR_WORKSPACE;
    *out = u->second.ptr;
    return UH_OK;
  }
  Workspace &w = g_lib_ws[std::make_pair(dev, stream)];
  if (w.bytes < need) {
    bool cap = false;
    int rc = capturing(stream, &cap);
    if (rc) return rc;
    if (cap) return UH_ERR_CAPTURE;
    // work already enqueued on this stream may still use the old memory:
    // hipFree waits for it
    if (w.ptr) (void)hipFree(w.ptr);
    w.ptr = nullptr;
    w.bytes = 0;
    const size_t want = std::max(need, (size_t)(1 << 20));
    if (hipMalloc(&w.ptr, want) != hipSuccess) {
      w.ptr = nullptr;
      return UH_ERR_ALLOC;
    }
    w.bytes = want;
  }
  *out = w.ptr;
  return UH_OK;
}

// One set of n points (with both hoods: its upper hood into out_idx[0 .. n),
// out_count[0], and its lower hood into out_idx[n .. 2n), out_count[1]; the
// hood buffers inside the workspace if hood_bufs is given).
// fixed != nullptr: the working memory is fixed[0 .. fixed_bytes) instead of
// a workspace (upper_hull_noalloc); a run that needs more is refused.
int run_single(const float *points, int64_t n, bool both, int32_t *out_idx, int32_t *out_count,
               hipStream_t stream, int32_t **hood_idx, int32_t **hood_cnt,
               void *fixed = nullptr, size_t fixed_bytes = 0) {
  const int K = 16;
  bool large = false;
  const int64_t off[2] = {0, n};
  const int cus = cu_count();
  const int F = default_fan_in(off, 1, 64 * K, cus, &large);
  SingleShape sh;
  single_shape(n, both, K, F, large, sh);
  const bool bufs = hood_idx != nullptr;
  const SingleLayout L = single_layout(sh, bufs);
  void *base = fixed;
  if (fixed) {
    if (L.total > fixed_bytes) return UH_ERR_TOO_LARGE;
  } else {
    const int rc = single_workspace(L.total, stream, &base);
    if (rc) return rc;
  }
  char *b = static_cast<char *>(base);
  if (bufs) {
    *hood_idx = reinterpret_cast<int32_t *>(b + L.hull_idx);
    *hood_cnt = reinterpret_cast<int32_t *>(b + L.hull_cnt);
    out_idx = *hood_idx;
    out_count = *hood_cnt;
  }
  if (n == 0) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, stream, out_count, sh.VS, 0);
    return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
  }
  Launch La;
  RunArgs &A = La.A;
  A.pts = reinterpret_cast<const float2 *>(points);
  A.set_start = nullptr;
  A.ws_xy = reinterpret_cast<float2 *>(b + L.ws_xy);
  A.ws_idx = reinterpret_cast<int32_t *>(b + L.ws_idx);
  A.set_status = reinterpret_cast<int32_t *>(b + L.status);
  A.out_idx = out_idx;
  A.out_counts = out_count;
  A.stats = nullptr;
  A.n_total = (int64_t)sh.VS * n;
  A.tile_len = sh.T;
  A.one_set = 1;
  A.group_fan = sh.group_fan;
  A.tile_max = reinterpret_cast<uint32_t *>(b + L.tile_max);
  A.group_max = reinterpret_cast<uint32_t *>(b + L.group_max);
  A.flags = both ? UH_FLAG_BOTH_HOODS : 0u;
  A.n_points = n;
  A.lower_n = both ? n : 0;
  A.lower_tiles = both ? sh.tiles : 0;
  A.lower_groups = both ? sh.groups : 0;
  A.lower_sets = both ? 1 : 0;
  La.S = sh.VS;
  La.tile_grid = sh.tiles;
  La.K = K;
  La.both = both;
  La.cnt0 = reinterpret_cast<int32_t *>(b + L.cnt0);
  La.npass = sh.npass;
  for (int k = 0; k < sh.npass; ++k) {
    La.pass_items[k] = sh.VS * sh.pass[k].items;
    La.pass_reps[k] = k + 1 == sh.npass ? last_pass_reps(La.pass_items[k], cus) : 1;
    La.pass_wide[k] = sh.wide[k];
    La.items[k] = nullptr;
    La.order[k] = nullptr;
    La.cnt[k] = reinterpret_cast<int32_t *>(b + L.cnt[k]);
    La.pa[k] = sh.pass[k];
  }
  // the workspace may hold anything from runs of other shapes: clear the
  // status and group maxima this run reads (a one-tile set reads neither)
  La.init = sh.tiles > 1;
  La.init_groups = sh.VS * sh.groups;
  return enqueue(La, stream);
}

// ---- fixed scratch of upper_hull_noalloc
// The working memory of upper_hull_noalloc: a device array of the library's
// own, sized for UH_NOALLOC_MAX_N points, one copy per device, held until the
// process ends.  Host code never passes its name to a kernel (on the host it
// is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_BYTES = workspace_bound((size_t)UH_NOALLOC_MAX_N, 1);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_DEVICES];  // device address of `scratch` per device (null: not yet)

// The current device's copy of `scratch`: its address is looked up on the
// device's first call and kept (no allocation: the array is part of the
// loaded code object).
int noalloc_scratch(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UH_ERR_HIP;
  if (dev < 0 || dev >= NOALLOC_DEVICES) return UH_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return UH_ERR_HIP;
    g_noalloc_ptr[dev] = ptr;
  }
  *out = g_noalloc_ptr[dev];
  return UH_OK;
}

// ---- cached plans of the batched call without a plan object
struct CachedPlan {
  upper_hull_plan *plan = nullptr;
  uint64_t last_use = 0;
  int in_use = 0;               // calls between taking the plan and enqueueing
  bool captured = false;        // used while a stream was capturing: never dropped
  hipEvent_t done = nullptr;    // recorded after its latest run
};
constexpr size_t BATCHED_CACHE = 8;
std::mutex g_cache_mu;
uint64_t g_clock = 0;
std::map<std::pair<int, std::vector<int64_t>>, CachedPlan> g_batched_plans;
std::vector<CachedPlan> g_retired;  // dropped, freed once their last run is done

// Frees retired plans whose last run has finished (never waits).
void reap_retired() {
  for (size_t k = 0; k < g_retired.size();) {
    CachedPlan &c = g_retired[k];
    if (!c.done || hipEventQuery(c.done) == hipSuccess) {
      if (c.done) (void)hipEventDestroy(c.done);
      upper_hull_plan *p = c.plan;
      int cur = 0;
      (void)hipGetDevice(&cur);
      (void)hipSetDevice(p->device);
      free_plan_memory(p);
      (void)hipSetDevice(cur);
      delete p;
      g_retired.erase(g_retired.begin() + (long)k);
    } else {
      ++k;
    }
  }
}

}  // namespace

extern "C" {

const char *upper_hull_status_string(int status) {
  switch (status) {
    case UH_OK: return "ok";
    case UH_ERR_ARG: return "invalid argument";
    case UH_ERR_ALLOC: return "device allocation failed";
    case UH_ERR_HIP: return "HIP runtime error";
    case UH_ERR_CAPTURE: return "allocation needed while the stream is capturing";
    case UH_ERR_WORKSPACE: return "the workspace set is too small for this call";
    case UH_ERR_TOO_LARGE: return "more points than upper_hull_noalloc's fixed scratch serves";
    case UH_ERR_UNSORTED: return "data error: x not non-decreasing";
    case UH_ERR_RANGE: return "data error: coordinate out of range or not finite";
    case UH_ERR_GRID: return "data error: coordinate not on the 2^-30 grid";
    default: return status >= 0 ? "ok (count)" : "unknown status";
  }
}

size_t upper_hull_workspace_bytes(int64_t max_total_n, int32_t max_sets) {
  if (max_total_n < 0 || max_sets < 1 || max_total_n > ((int64_t)1 << 40)) return 0;
  return workspace_bound((size_t)max_total_n, (size_t)max_sets);
}

int upper_hull_set_workspace(void *device_ptr, size_t bytes) {
  if ((device_ptr == nullptr) != (bytes == 0)) return UH_ERR_ARG;
  if (((uintptr_t)device_ptr & 255u) != 0) return UH_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UH_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_ws_mu);
  if (device_ptr)
    g_user_ws[dev] = Workspace{device_ptr, bytes};
  else
    g_user_ws.erase(dev);
  return UH_OK;
}

int upper_hull_plan_create(const int64_t *set_offsets, int32_t num_sets,
                           const upper_hull_config *config,
                           upper_hull_plan **out_plan) {
  if (!set_offsets || num_sets < 1 || !out_plan) return UH_ERR_ARG;
  *out_plan = nullptr;
  if (set_offsets[0] != 0) return UH_ERR_ARG;
  for (int32_t s = 0; s < num_sets; ++s) {
    if (set_offsets[s + 1] < set_offsets[s]) return UH_ERR_ARG;
    if (set_offsets[s + 1] - set_offsets[s] > INT32_MAX) return UH_ERR_ARG;
  }
  int K = 16, F = 0;
  uint32_t flags = 0;
  if (config) {
    if (config->strip) K = config->strip;
    F = config->fan_in;
    flags = config->flags;
  }
  if (K != 4 && K != 8 && K != 16 && K != 32) return UH_ERR_ARG;
  if (F != 0 && (F < 2 || F > BLOCK || (F & (F - 1)))) return UH_ERR_ARG;
  bool large_plan = false;
  const int Fdef = default_fan_in(set_offsets, num_sets, 64 * K, cu_count(), &large_plan);
  if (F == 0) F = Fdef;
  // the sort's positions are 32-bit
  if ((flags & UH_FLAG_UNSORTED) && set_offsets[num_sets] > (int64_t)UINT32_MAX) return UH_ERR_ARG;

  // With both hoods the schedule covers 2 * num_sets sets over 2 * N slots:
  // set num_sets + s is the lower hood of set s (the mirrored points), its
  // slots and outputs N further on.  Its tiles and groups mirror those of
  // set s, since sets are laid out in order and the two halves are alike.
  const bool both = (flags & UH_FLAG_BOTH_HOODS) != 0;
  const int32_t VS = both ? 2 * num_sets : num_sets;
  std::vector<int64_t> voff(set_offsets, set_offsets + num_sets + 1);
  if (both)
    for (int32_t s = 0; s < num_sets; ++s) voff.push_back(set_offsets[num_sets] + set_offsets[s + 1]);
  auto *p = new upper_hull_plan();
  (void)hipGetDevice(&p->device);
  p->both = both;
  p->in_S = num_sets;
  p->in_N = set_offsets[num_sets];
  p->S = VS;
  p->N = voff[VS];
  p->K = K;
  p->T = 64 * K;
  p->F = F;
  p->flags = flags;
  for (int32_t s = 0; s < VS; ++s) p->has_empty = p->has_empty || voff[s + 1] == voff[s];

  std::vector<TileItem> tiles;
  std::vector<std::vector<MergeItem>> passes;
  if (num_sets == 1) {
    // one set: every tile and merge item follows from its index
    single_shape(p->in_N, both, K, F, large_plan, p->single);
    const SingleShape &sh = p->single;
    p->ntiles = sh.VS * sh.tiles;
    p->ngroups = sh.VS * sh.groups;
    p->group_fan = sh.group_fan;
    for (int k = 0; k < sh.npass; ++k) {
      p->pass_items.push_back(sh.VS * sh.pass[k].items);
      p->pass_wide.push_back(sh.wide[k]);
    }
  } else {
    // level 0: tiles; then merge passes of fan-in F until one hood per set
    std::vector<int32_t> first(VS), count(VS);  // blocks per set
    for (int32_t s = 0; s < VS; ++s) {
      const int64_t n = voff[s + 1] - voff[s];
      const int64_t nt = (n + p->T - 1) / p->T;
      first[s] = (int32_t)tiles.size();
      count[s] = (int32_t)nt;
      for (int64_t t = 0; t < nt; ++t) {
        TileItem it;
        it.start = voff[s] + t * p->T;
        it.len = (int32_t)std::min<int64_t>(p->T, n - t * p->T);
        it.set = s;
        it.rel0 = (int32_t)(t * p->T);
        it.nb_lo = (int16_t)std::min<int64_t>(16, t * p->T);
        it.nb_hi = (int16_t)std::min<int64_t>(16, n - t * p->T - it.len);
        it.set_len = (int32_t)n;
        it.group = -1;  // set below, once the first merge level is known
        tiles.push_back(it);
      }
    }
    p->ntiles = (int32_t)tiles.size();
    // Within a set the blocks of a level are consecutive and equally long
    // (except the last), so child k of an item starts at off + k * stride.
    std::vector<int32_t> g0(VS, 0), ng(VS, 0), fs0(VS, F);  // first level per set
    int64_t stride = p->T;
    for (;;) {
      std::vector<MergeItem> items;
      std::vector<int32_t> nfirst(VS), ncount(VS);
      // With the default fan-in, a set with BLOCK + 1 .. WIDE blocks left can
      // finish in one wide workgroup (one per CU), if few sets need one.
      int32_t nwide = 0;
      for (int32_t s = 0; s < VS; ++s) nwide += F == BLOCK && count[s] > BLOCK && count[s] <= WIDE;
      const bool use_wide = nwide > 0 && nwide <= 256;
      for (int32_t s = 0; s < VS; ++s) {
        nfirst[s] = (int32_t)items.size();
        ncount[s] = 0;
        if (count[s] <= 1) continue;
        const int32_t FS = use_wide && F == BLOCK && count[s] <= WIDE ? WIDE : F;
        const int32_t nitems = (count[s] + FS - 1) / FS;
        for (int32_t i = 0; i < nitems; ++i) {
          MergeItem m;
          m.child0 = first[s] + i * FS;
          m.nch = std::min(FS, count[s] - i * FS);
          m.off = voff[s] + (int64_t)i * FS * stride;
          m.stride = stride;
          m.set = s;
          m.final_ = nitems == 1;
          m.level = std::min<int32_t>((int32_t)passes.size(), 2);
          m.g0 = m.ng = m.pad = 0;
          items.push_back(m);
        }
        ncount[s] = nitems;
        if (passes.empty()) {
          g0[s] = nfirst[s];
          ng[s] = nitems;
          fs0[s] = FS;
        }
      }
      if (items.empty()) break;
      passes.push_back(items);
      stride *= F;
      first = nfirst;
      // sets finished in this pass keep count 1 -> no further items
      for (int32_t s = 0; s < VS; ++s) count[s] = ncount[s];
    }
    // groups: the first-level items; every item knows its set's groups, and
    // every tile of a set with more than one tile knows its group
    for (auto &items : passes)
      for (MergeItem &m : items) {
        m.g0 = g0[m.set];
        m.ng = ng[m.set];
      }
    for (int32_t s = 0, t0 = 0; s < VS; ++s) {
      const int64_t n = voff[s + 1] - voff[s];
      const int32_t nt = (int32_t)((n + p->T - 1) / p->T);
      if (nt > 1)
        for (int32_t t = 0; t < nt; ++t) tiles[t0 + t].group = g0[s] + t / fs0[s];
      t0 += nt;
    }
    p->group_fan = fs0[0];
    p->ngroups = passes.empty() ? 0 : (int32_t)passes[0].size();
    if (both) {
      // the tile kernel derives each lower tile from its upper twin: check that
      // the schedule's second half is the first half moved by (N, S, tiles/2,
      // groups/2), which holds because the two halves have the same set sizes
      const int32_t ht = p->ntiles / 2, hg = p->ngroups / 2;
      bool ok = p->ntiles % 2 == 0 && p->ngroups % 2 == 0;
      for (int32_t t = 0; ok && t < ht; ++t) {
        const TileItem &a = tiles[t], &b = tiles[t + ht];
        ok = b.start == a.start + p->in_N && b.len == a.len && b.set == a.set + num_sets &&
             b.rel0 == a.rel0 && b.nb_lo == a.nb_lo && b.nb_hi == a.nb_hi &&
             b.set_len == a.set_len && b.group == (a.group < 0 ? -1 : a.group + hg);
      }
      if (!ok) {
        delete p;
        return UH_ERR_ARG;
      }
    }
    for (auto &items : passes) {
      p->pass_items.push_back((int32_t)items.size());
      bool wide = large_plan && items.size() <= 64;
      for (const MergeItem &m : items) wide = wide || m.nch > BLOCK;
      p->pass_wide.push_back(wide);
    }
  }
  if (!p->pass_items.empty()) p->last_reps = last_pass_reps(p->pass_items.back(), cu_count());
  p->h_voff = voff;
  p->h_tiles = tiles;
  p->h_items = passes;
  int rc = UH_OK;
  std::vector<int64_t> so(voff.begin(), voff.end());
  rc = rc ? rc : dalloc(&p->d_set_start, so.size());
  rc = rc ? rc : upload(p->d_set_start, so);
  if (!tiles.empty()) {
    rc = rc ? rc : dalloc(&p->d_tiles, tiles.size());
    rc = rc ? rc : upload(p->d_tiles, tiles);
  }
  rc = rc ? rc : dalloc(&p->d_cnt0, (size_t)p->ntiles);
  for (size_t k = 0; k < p->pass_items.size(); ++k) {
    if (rc) break;
    if (!passes.empty()) {
      MergeItem *di = nullptr;
      rc = rc ? rc : dalloc(&di, passes[k].size());
      rc = rc ? rc : upload(di, passes[k]);
      p->d_items.push_back(di);
      // launch order: the items with the most children first, so that the
      // largest merges of a batch do not start last and leave a tail
      std::vector<int32_t> ord(passes[k].size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int32_t)i;
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        return passes[k][(size_t)a].nch > passes[k][(size_t)b].nch;
      });
      bool identity = true;
      for (size_t i = 0; i < ord.size(); ++i) identity = identity && ord[i] == (int32_t)i;
      int32_t *dord = nullptr;
      if (!identity) {
        rc = rc ? rc : dalloc(&dord, ord.size());
        rc = rc ? rc : upload(dord, ord);
      }
      p->d_order.push_back(dord);
    }
    int32_t *dcnt = nullptr;
    rc = rc ? rc : dalloc(&dcnt, (size_t)p->pass_items[k]);
    p->d_cnt.push_back(dcnt);
  }
  if (!rc && (flags & UH_FLAG_UNSORTED)) {
    p->unsorted = true;
    rc = uh_rs::radix_plan_build(set_offsets, num_sets, &p->rs);
    rc = rc ? rc : dalloc(&p->sorted, (size_t)p->in_N);
    rc = rc ? rc : dalloc(&p->perm, (size_t)p->in_N);
  }
  rc = rc ? rc : dalloc(&p->ws_xy, (size_t)p->N);
  rc = rc ? rc : dalloc(&p->ws_idx, (size_t)p->N);
  rc = rc ? rc : dalloc(&p->set_status, (size_t)VS);
  rc = rc ? rc : dalloc(&p->tile_max, (size_t)p->ntiles);
  rc = rc ? rc : dalloc(&p->group_max, (size_t)p->ngroups * GROUP_STRIDE);
  if (!rc && p->ngroups > 0 &&
      hipMemset(p->group_max, 0, (size_t)p->ngroups * GROUP_STRIDE * sizeof(uint32_t)) !=
          hipSuccess)
    rc = UH_ERR_HIP;
  if (!rc && hipMemset(p->set_status, 0, (size_t)VS * sizeof(int32_t)) != hipSuccess)
    rc = UH_ERR_HIP;
  if (rc) {
    free_plan_memory(p);
    delete p;
    return rc;
  }
  *out_plan = p;
  return UH_OK;
}

int upper_hull_plan_sorted(const upper_hull_plan *plan, const float **sorted_points,
                           const int32_t **perm) {
  if (!plan || !plan->unsorted || !sorted_points || !perm) return UH_ERR_ARG;
  *sorted_points = (const float *)plan->sorted;
  *perm = plan->perm;
  return UH_OK;
}

int upper_hull_plan_config(const upper_hull_plan *plan, upper_hull_config *config) {
  if (!plan || !config) return UH_ERR_ARG;
  config->strip = plan->K;
  config->fan_in = plan->F;
  config->flags = plan->flags;
  return UH_OK;
}

int upper_hull_plan_launches(const upper_hull_plan *plan, int32_t with_stats) {
  if (!plan) return UH_ERR_ARG;
  const int sort = plan->unsorted && plan->rs.nblocks > 0 ? 5 * uh_rs::RS_PASSES : 0;
  return sort + (int)(plan->has_empty || with_stats) + (plan->ntiles > 0) +
         (int)plan->pass_items.size() + (plan->unsorted ? 1 : 0);
}

int upper_hull_plan_set_probe(upper_hull_plan *plan, hipEvent_t before,
                              hipEvent_t after) {
  if (!plan || (plan->flags & UH_FLAG_GRAPH) || (!before) != (!after)) return UH_ERR_ARG;
  plan->probe_before = before;
  plan->probe_after = after;
  return UH_OK;
}

int upper_hull_plan_run(upper_hull_plan *p, const float *points, int32_t *out_idx,
                        int32_t *out_counts, upper_hull_stats *stats,
                        hipStream_t stream) {
  if (!p || !out_counts || (p->N > 0 && (!points || !out_idx))) return UH_ERR_ARG;
  if (((uintptr_t)points & 7u) != 0) return UH_ERR_ARG;
  RunArgs A;
  A.pts = (const float2 *)points;
  A.set_start = p->d_set_start;
  A.ws_xy = p->ws_xy;
  A.ws_idx = p->ws_idx;
  A.set_status = p->set_status;
  A.out_idx = out_idx;
  A.out_counts = out_counts;
  A.stats = stats;
  A.n_total = p->N;
  A.tile_len = p->T;
  A.group_fan = p->group_fan;
  A.tile_max = p->tile_max;
  A.group_max = p->group_max;
  A.one_set = p->in_S == 1;
  A.flags = p->flags;
  A.n_points = p->in_N;
  A.lower_n = p->both ? p->in_N : 0;
  A.lower_tiles = p->both ? p->ntiles / 2 : 0;
  A.lower_groups = p->both ? p->ngroups / 2 : 0;
  A.lower_sets = p->both ? p->in_S : 0;
  if (!(p->flags & UH_FLAG_GRAPH)) return enqueue_run(p, A, stream);

  std::lock_guard<std::mutex> lock(p->mu);
  const auto key = std::make_tuple((const void *)points, (void *)out_idx, (void *)out_counts,
                                   (void *)stats);
  size_t at = p->graphs.size();
  for (size_t k = 0; k < p->graphs.size(); ++k)
    if (p->graphs[k].first == key) at = k;
  if (at == p->graphs.size()) {
    if (!p->cap_stream &&
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return UH_ERR_HIP;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
      return UH_ERR_HIP;
    const int rc = enqueue_run(p, A, p->cap_stream);
    if (hipStreamEndCapture(p->cap_stream, &g) != hipSuccess || rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : UH_ERR_HIP;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return UH_ERR_HIP;
    if (p->graphs.size() >= upper_hull_plan::GRAPH_CACHE) {  // drop the least recently used
      // its earlier launches are ordered before this run's on their streams;
      // destroying the executable does not cancel them
      (void)hipGraphExecDestroy(p->graphs.front().second);
      p->graphs.erase(p->graphs.begin());
    }
    p->graphs.emplace_back(key, ex);
    at = p->graphs.size() - 1;
  } else if (at + 1 != p->graphs.size()) {  // most recently used goes last
    auto e = p->graphs[at];
    p->graphs.erase(p->graphs.begin() + (long)at);
    p->graphs.push_back(e);
    at = p->graphs.size() - 1;
  }
  return hipGraphLaunch(p->graphs[at].second, stream) == hipSuccess ? UH_OK : UH_ERR_HIP;
}

int32_t upper_hull_plan_blocks(const upper_hull_plan *p, int32_t level, int64_t *ranges) {
  if (!p || level < 0 || level > (int32_t)p->pass_items.size()) return UH_ERR_ARG;
  const int32_t nb = level == 0 ? p->ntiles : p->pass_items[level - 1];
  if (!ranges) return nb;
  for (int32_t b = 0; b < nb; ++b) {
    int64_t start, end;
    if (p->in_S == 1) {
      const SingleShape &sh = p->single;
      if (level == 0) {
        const int32_t v = b / sh.tiles, t = b - v * sh.tiles;
        start = v * sh.n + (int64_t)t * sh.T;
        end = std::min(start + sh.T, (v + 1) * sh.n);
      } else {
        const PassArgs &pa = sh.pass[level - 1];
        const int32_t v = b / pa.items, i = b - v * pa.items;
        start = v * sh.n + (int64_t)i * pa.fan * pa.stride;
        end = std::min(start + (int64_t)pa.fan * pa.stride, (v + 1) * sh.n);
      }
    } else if (level == 0) {
      start = p->h_tiles[b].start;
      end = start + p->h_tiles[b].len;
    } else {
      const MergeItem &m = p->h_items[level - 1][b];
      start = m.off;
      end = std::min(m.off + (int64_t)m.nch * m.stride, p->h_voff[m.set + 1]);
    }
    ranges[2 * b] = start;
    ranges[2 * b + 1] = end - start;
  }
  return nb;
}

int upper_hull_plan_trace(upper_hull_plan *p, const float *points, int32_t level,
                          int32_t *out_idx, int32_t *out_counts, hipStream_t stream) {
  if (!p || p->unsorted || !out_counts || level < 0 ||
      level > (int32_t)p->pass_items.size() || (p->N > 0 && (!points || !out_idx)))
    return UH_ERR_ARG;
  if (((uintptr_t)points & 7u) != 0) return UH_ERR_ARG;
  if (!p->trace_cnt) {
    bool cap = false;
    int rc = capturing(stream, &cap);
    if (rc) return rc;
    if (cap) return UH_ERR_CAPTURE;
    rc = dalloc(&p->trace_cnt, (size_t)p->S);
    if (rc) return rc;
  }
  RunArgs A;
  A.pts = (const float2 *)points;
  A.set_start = p->d_set_start;
  A.ws_xy = p->ws_xy;
  A.ws_idx = p->ws_idx;
  A.set_status = p->set_status;
  A.out_idx = out_idx;
  A.out_counts = p->trace_cnt;
  A.stats = nullptr;
  A.n_total = p->N;
  A.tile_len = p->T;
  A.group_fan = p->group_fan;
  A.tile_max = p->tile_max;
  A.group_max = p->group_max;
  A.one_set = p->in_S == 1;
  A.flags = p->flags;
  A.n_points = p->in_N;
  A.lower_n = p->both ? p->in_N : 0;
  A.lower_tiles = p->both ? p->ntiles / 2 : 0;
  A.lower_groups = p->both ? p->ngroups / 2 : 0;
  A.lower_sets = p->both ? p->in_S : 0;
  Launch L = plan_launch(p, A, false);
  L.npass = level;  // the tile pass and merge passes 1 .. level
  L.probe_before = L.probe_after = nullptr;
  int rc = enqueue(L, stream);
  if (rc) return rc;
  if (level < (int32_t)p->pass_items.size()) {
    // the next pass reads the group maxima of this run: it would have cleared
    // them at its sets' final merges, so clear them here
    Launch Z = L;
    Z.tile_grid = 0;
    Z.npass = 0;
    Z.init = true;
    Z.init_groups = p->ngroups;
    Z.A.out_counts = p->trace_cnt;
    // (init also resets the run's status and the counts of empty sets)
    const int32_t nb = level == 0 ? p->ntiles : p->pass_items[level - 1];
    const PassArgs pa = level == 0 || p->in_S != 1 ? PassArgs{} : p->single.pass[level - 1];
    const MergeItem *items = level == 0 || p->d_items.empty() ? nullptr : p->d_items[level - 1];
    const int32_t *cnt = level == 0 ? p->d_cnt0 : p->d_cnt[level - 1];
    hipLaunchKernelGGL(trace_kernel, dim3((unsigned)std::max(nb, 1)), dim3(64), 0, stream, A,
                       level, p->in_S == 1 ? p->single.tiles : 0, p->d_tiles, items, pa, cnt,
                       out_counts);
    if (hipGetLastError() != hipSuccess) return UH_ERR_HIP;
    return enqueue(Z, stream);
  }
  const int32_t nb = p->pass_items.empty() ? p->ntiles : p->pass_items.back();
  const PassArgs pa = level == 0 || p->in_S != 1 ? PassArgs{} : p->single.pass[level - 1];
  const MergeItem *items = level == 0 || p->d_items.empty() ? nullptr : p->d_items[level - 1];
  const int32_t *cnt = level == 0 ? p->d_cnt0 : p->d_cnt[level - 1];
  if (nb > 0)
    hipLaunchKernelGGL(trace_kernel, dim3((unsigned)nb), dim3(64), 0, stream, A, level,
                       p->in_S == 1 ? p->single.tiles : 0, p->d_tiles, items, pa, cnt,
                       out_counts);
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

void upper_hull_plan_destroy(upper_hull_plan *plan) {
  if (!plan) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(plan->device);
  (void)hipDeviceSynchronize();
  free_plan_memory(plan);
  (void)hipSetDevice(cur);
  delete plan;
}

int upper_hull(const float *points, int64_t n, int32_t *out_idx, int32_t *out_count,
               hipStream_t stream) {
  if (n < 0 || n > INT32_MAX || !out_count || (n > 0 && (!points || !out_idx)))
    return UH_ERR_ARG;
  if (((uintptr_t)points & 7u) != 0) return UH_ERR_ARG;
  return run_single(points, n, false, out_idx, out_count, stream, nullptr, nullptr);
}

int upper_hull_noalloc(const float *points, int64_t n, int32_t *out_idx, int32_t *out_count,
                       hipStream_t stream) {
  if (n < 0 || !out_count || (n > 0 && (!points || !out_idx))) return UH_ERR_ARG;
  if (n > UH_NOALLOC_MAX_N) return UH_ERR_TOO_LARGE;
  if (((uintptr_t)points & 7u) != 0) return UH_ERR_ARG;
  void *ptr = nullptr;
  const int rc = noalloc_scratch(&ptr);
  if (rc) return rc;
  return run_single(points, n, false, out_idx, out_count, stream, nullptr, nullptr, ptr,
                    NOALLOC_BYTES);
}

int convex_hull(const float *points, int64_t n, int32_t *out_idx, int32_t *out_count,
                hipStream_t stream) {
  if (n < 0 || n > INT32_MAX || !out_count || (n > 0 && (!points || !out_idx)))
    return UH_ERR_ARG;
  if (((uintptr_t)points & 7u) != 0) return UH_ERR_ARG;
  // both hoods into buffers in the workspace, then one join pass into out_idx
  int32_t *hood_idx = nullptr, *hood_cnt = nullptr;
  int rc = run_single(points, n, true, nullptr, nullptr, stream, &hood_idx, &hood_cnt);
  if (rc) return rc;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(hull_assemble_kernel, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(256),
                     0, stream, hood_idx, hood_cnt, n, out_idx, out_count);
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

int upper_hull_batched(const float *points, const int64_t *set_offsets, int32_t num_sets,
                       int32_t *out_idx, int32_t *out_counts, upper_hull_stats *stats,
                       hipStream_t stream) {
  if (!set_offsets || num_sets < 1 || !out_counts) return UH_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UH_ERR_HIP;
  bool cap = false;
  int rc = capturing(stream, &cap);
  if (rc) return rc;
  CachedPlan *cp = nullptr;
  auto key = std::make_pair(dev, std::vector<int64_t>(set_offsets, set_offsets + num_sets + 1));
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (!cap) reap_retired();
    auto it = g_batched_plans.find(key);
    if (it == g_batched_plans.end()) {
      if (cap) return UH_ERR_CAPTURE;
      if (g_batched_plans.size() >= BATCHED_CACHE) {
        // drop the least recently used layout that no call is using and no
        // captured graph refers to; its memory is freed once its last run is done
        auto victim = g_batched_plans.end();
        for (auto v = g_batched_plans.begin(); v != g_batched_plans.end(); ++v)
          if (v->second.in_use == 0 && !v->second.captured &&
              (victim == g_batched_plans.end() || v->second.last_use < victim->second.last_use))
            victim = v;
        if (victim != g_batched_plans.end()) {
          g_retired.push_back(victim->second);
          g_batched_plans.erase(victim);
          reap_retired();
        }
      }
      upper_hull_plan *p = nullptr;
      rc = upper_hull_plan_create(set_offsets, num_sets, nullptr, &p);
      if (rc) return rc;
      it = g_batched_plans.emplace(std::move(key), CachedPlan{p}).first;
    }
    cp = &it->second;
    cp->last_use = ++g_clock;
    ++cp->in_use;
    cp->captured = cp->captured || cap;
  }
  rc = upper_hull_plan_run(cp->plan, points, out_idx, out_counts, stats, stream);
  std::lock_guard<std::mutex> lock(g_cache_mu);
  if (!rc && !cap) {
    if (!cp->done && hipEventCreateWithFlags(&cp->done, hipEventDisableTiming) != hipSuccess)
      cp->done = nullptr;
    if (cp->done && hipEventRecord(cp->done, stream) != hipSuccess) {
      (void)hipEventDestroy(cp->done);
      cp->done = nullptr;
    }
  }
  --cp->in_use;
  return rc;
}

int upper_hull_autotune(const float *points, const int64_t *set_offsets,
                        int32_t num_sets, uint32_t flags, int32_t reps,
                        upper_hull_config *best, float *best_ms,
                        hipStream_t stream) {
  if (!set_offsets || num_sets < 1 || !best || reps < 1 || reps > 1000) return UH_ERR_ARG;
  const int64_t N = set_offsets[num_sets];
  if (N > 0 && !points) return UH_ERR_ARG;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return UH_ERR_HIP;
  if (cs != hipStreamCaptureStatusNone) return UH_ERR_CAPTURE;
  flags &= ~UH_FLAG_GRAPH;
  int32_t *out_idx = nullptr, *out_counts = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int h = (flags & UH_FLAG_BOTH_HOODS) ? 2 : 1;  // hoods per set
  int rc = dalloc(&out_idx, (size_t)std::max<int64_t>(h * N, 1));
  rc = rc ? rc : dalloc(&out_counts, (size_t)(h * num_sets));
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = UH_ERR_HIP;
  float best_t = -1.0f;
  upper_hull_config chosen = {16, 256, flags};
  static const int strips[] = {8, 16, 32}, fans[] = {16, 32, 64, 128, 256};
  for (int si = 0; si < 3 && !rc; ++si) {
    for (int fi = 0; fi < 5 && !rc; ++fi) {
      const upper_hull_config cfg = {strips[si], fans[fi], flags};
      upper_hull_plan *plan = nullptr;
      rc = upper_hull_plan_create(set_offsets, num_sets, &cfg, &plan);
      if (rc) break;
      rc = upper_hull_plan_run(plan, points, out_idx, out_counts, nullptr, stream);  // untimed
      if (!rc && hipEventRecord(e0, stream) != hipSuccess) rc = UH_ERR_HIP;
      for (int r = 0; r < reps && !rc; ++r)
        rc = upper_hull_plan_run(plan, points, out_idx, out_counts, nullptr, stream);
      float ms = 0.0f;
      if (!rc && (hipEventRecord(e1, stream) != hipSuccess ||
                  hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = UH_ERR_HIP;
      upper_hull_plan_destroy(plan);
      ms /= (float)reps;
      if (!rc && (best_t < 0.0f || ms < best_t)) {
        best_t = ms;
        chosen = cfg;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out_idx);
  (void)hipFree(out_counts);
  if (rc) return rc;
  *best = chosen;
  if (best_ms) *best_ms = best_t;
  return UH_OK;
}

int upper_hull_bridge(const float *P, int32_t hp, const float *Q, int32_t hq,
                      int32_t lanes, int32_t *out_ab, hipStream_t stream) {
  if (!P || !Q || !out_ab || hp < 1 || hq < 1) return UH_ERR_ARG;
  if (lanes < 1 || lanes > 64 || (lanes & (lanes - 1))) return UH_ERR_ARG;
  hipLaunchKernelGGL(bridge_kernel, dim3(1), dim3(64), 0, stream, (const float2 *)P, hp,
                     (const float2 *)Q, hq, lanes, out_ab);
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

int upper_hull_orient(const float *a, const float *b, const float *c, int64_t m,
                      int8_t *out_sign, uint8_t *out_fallback, int32_t force_fallback,
                      hipStream_t stream) {
  if (m < 0 || (m > 0 && (!a || !b || !c || !out_sign))) return UH_ERR_ARG;
  if (m == 0) return UH_OK;
  const int64_t nb = (m + 255) / 256;
  if (nb > INT32_MAX) return UH_ERR_ARG;
  hipLaunchKernelGGL(orient_kernel, dim3((unsigned)nb), dim3(256), 0, stream,
                     (const float2 *)a, (const float2 *)b, (const float2 *)c, m, out_sign,
                     out_fallback, force_fallback);
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

}  // extern "C"
