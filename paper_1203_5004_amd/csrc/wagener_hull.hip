// wagener_hull.hip -- kernels, schedule and C ABI of the upper-hood library.
//
// Paper: C. O Dunlaing, "CUDA implementation of Wagener's 2D convex hull PRAM
// algorithm".  The paper's program copies the padded hood array to the GPU,
// launches match_and_merge once per stage (d = 2, 4, ..., n/2) and copies it
// back after every stage.  Here the same rounds of pairwise hood merges run
// device-resident, in three kinds of launch enqueued back to back:
//
//   init_kernel   clears per-set status and counters.
//   tile_kernel   one workgroup per tile of T = 256 * K points of one set:
//                 coalesced load (plus contract checks) into LDS; each lane
//                 builds the hood of its strip of K consecutive points
//                 serially (the first step of the paper's work-optimal
//                 variant in its conclusions); then log2(256) = 8 rounds of
//                 Wagener merges of adjacent strip hoods in LDS, each merge
//                 finding its bridge with the sampled search of one wave and
//                 compacting P[0..a] ++ Q[b..]; the tile hood goes to the
//                 workspace (or straight to the output for a one-tile set).
//   merge_kernel  one workgroup merges up to F consecutive hoods of the
//                 previous level of one set through log2(F) further rounds,
//                 in LDS when they fit, else in place in the workspace.
//                 Repeated until every set has a single hood.
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

#include "uh_device.hpp"
#include "wagener_hull.h"

namespace uh {

constexpr int BLOCK = 256;       // threads per workgroup (4 waves)
constexpr int VMAX = 8192;       // corners a merge workgroup keeps in LDS
// Bit 31 of a tile's output count: the tile wrote its surviving points (a
// sorted point list, not yet a hood); the merge kernel makes it a hood.
constexpr uint32_t POINTS_FLAG = 0x80000000u;
constexpr int TILE_LIST_MAX = 64;  // most survivors a tile hands on as a list

struct TileItem {    // one tile of the tile pass
  int64_t start;     // first point (absolute)
  int32_t len;       // points, 1 .. T
  int32_t set;
  int32_t final_;    // 1 if this tile is its set's only tile
  int32_t pad;
};

struct MergeItem {   // one workgroup of a merge pass
  int64_t off;       // slot start = first child's slot start (absolute)
  int32_t child0;    // first child in the previous level's arrays
  int32_t nch;       // children, 2 .. F
  int32_t set;
  int32_t final_;    // 1 if this is its set's last merge
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
  uint32_t flags;
};

// ------------------------------------------------------------ small helpers
__device__ __forceinline__ int check_point(float2 v) {
  // data contract: x in [0,1], y in [-1,1] (NaN fails both), both on the
  // 2^-30 grid: scaling by 2^30 is exact, and then no fraction may remain
  if (!(__builtin_fabsf(v.x - 0.5f) <= 0.5f && __builtin_fabsf(v.y) <= 1.0f))
    return UH_ERR_RANGE;
  const float fr = __builtin_amdgcn_fractf(v.x * 0x1p30f) + __builtin_amdgcn_fractf(v.y * 0x1p30f);
  return fr == 0.0f ? 0 : UH_ERR_GRID;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds the workgroup's orientation counters to stats[set] (if any).
__device__ __forceinline__ void flush_stats(const RunArgs &A, int set,
                                            const OrientCount &oc,
                                            unsigned long long *sstat) {
  const uint32_t e = wave_sum(oc.evals), f = wave_sum(oc.fallbacks);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&sstat[0], (unsigned long long)e);
    atomicAdd(&sstat[1], (unsigned long long)f);
  }
  __syncthreads();
  if (threadIdx.x == 0 && A.stats) {
    atomicAdd((unsigned long long *)&A.stats[set].orient_evals, sstat[0]);
    atomicAdd((unsigned long long *)&A.stats[set].fallbacks, sstat[1]);
  }
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

// ---------------------------------------------------------------- init
__global__ void init_kernel(int32_t S, RunArgs A) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  A.set_status[s] = 0;
  if (A.stats) {
    A.stats[s].orient_evals = 0;
    A.stats[s].fallbacks = 0;
  }
  if (A.set_start[s + 1] == A.set_start[s]) A.out_counts[s] = 0;
}

// ---------------------------------------------------------------- tiles
// Workgroup barrier that orders LDS only: unlike __syncthreads it does not
// wait for outstanding global loads, so a prefetch stays in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave-level inclusive max scans (prefix: lanes below; suffix: lanes above).
__device__ __forceinline__ float wave_prefix_max(float v) {
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    const float y = __shfl_up(v, o, 64);
    if (lane >= o) v = fmaxf(v, y);
  }
  return v;
}
__device__ __forceinline__ float wave_suffix_max(float v) {
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    const float y = __shfl_down(v, o, 64);
    if (lane + o < 64) v = fmaxf(v, y);
  }
  return v;
}

// Adds a wave's orientation counters to stats[set].
__device__ __forceinline__ void flush_wave_stats(const RunArgs &A, int set, OrientCount &oc) {
  if (!A.stats) return;
  const uint32_t e = wave_sum(oc.evals), f = wave_sum(oc.fallbacks);
  if ((threadIdx.x & 63) == 0 && A.stats && e) {
    atomicAdd((unsigned long long *)&A.stats[set].orient_evals, (unsigned long long)e);
    atomicAdd((unsigned long long *)&A.stats[set].fallbacks, (unsigned long long)f);
  }
  oc.evals = oc.fallbacks = 0;
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// Tile kernel: one wave (one workgroup of 64 lanes) per tile of up to
// T = 64 * K points of one set; no workgroup barrier anywhere.
//  1. coalesced 16-byte loads (two points per lane per load), the data
//     contract's range and grid checks, then the points go to per-lane
//     strips of K consecutive points in LDS (stride K + 2: 16-byte aligned)
//     and each lane reads its strip back into registers;
//  2. strip pass 1: maximum y of each strip, x non-decreasing check (the
//     previous strip's last point comes from the neighbouring lane); wave
//     prefix and suffix maxima over the strips;
//  3. strip pass 2: exact elimination, then the strip hood.  A point r is
//     dropped when some earlier point of the tile is at least as high and
//     some later point is strictly higher: r then lies below the segment
//     joining the first earlier maximum and the last later maximum (both of
//     which survive), or directly below a point at its x, so it is no corner
//     of the tile's hood (nor is any identical copy of it that survives only
//     because it comes later).  The survivors go through a serial monotone
//     chain whose stack lives in the strip's LDS slot (the serial strip
//     hoods of the paper's work-optimal variant);
//  4. six rounds of Wagener merges (match-and-merge on adjacent hoods,
//     block size K * 2^j -> K * 2^(j+1)), the 2^(j+1) lanes of each merge
//     acting as the paper's d1 x d2 thread block;
//  5. the tile's hood goes to the workspace, or to the output for a
//     one-tile set.
template <int K>
__global__ __launch_bounds__(64) void tile_kernel(RunArgs A, const TileItem *items,
                                                  int32_t *cnt_out) {
  constexpr int S = K + 2;
  constexpr int NV = K / 2;  // 16-byte slots (point pairs) per lane
  __shared__ __attribute__((aligned(16))) float2 sxy[64 * S];
  __shared__ uint16_t sid[64 * S];
  __shared__ int2 sblk[64];  // (base, count) of the block starting at each strip

  const TileItem it = items[blockIdx.x];
  const int lane = threadIdx.x;
  const bool fe = (A.flags & UH_FLAG_FORCE_FALLBACK) != 0;
  const bool validate = (A.flags & UH_FLAG_NO_VALIDATE) == 0;
  const int64_t sstart = A.set_start[it.set];
  const float2 *src = A.pts + it.start;

  // ---- 1. load
  float4 v[NV];
  int err = 0;
  float prev_tile_x = -1.0f;  // below every valid x
  if (validate && lane == 0 && it.start > sstart) prev_tile_x = A.pts[it.start - 1].x;
  // Witnesses from the neighbouring tiles of the same set: the maximum y of
  // up to 16 points just before the tile and of up to 16 just after it
  // (lanes 0-15 fetch them, two points each).  Any earlier / later point of
  // the set may serve the elimination test below, and these let the first
  // and last strips drop their points too.
  float nb_before = -2.0f, nb_after = -2.0f;
  {
    const int64_t send = A.set_start[it.set + 1];
    float wy = -2.0f;
    if (lane < 8) {
      const int64_t e = it.start - 16 + 2 * lane;
      if (e >= sstart) wy = fmaxf(A.pts[e].y, A.pts[e + 1].y);
    } else if (lane < 16) {
      const int64_t e = it.start + it.len + 2 * (lane - 8);
      if (e + 1 < send) wy = fmaxf(A.pts[e].y, A.pts[e + 1].y);
      else if (e < send) wy = A.pts[e].y;
    }
    for (int o = 4; o > 0; o >>= 1) wy = fmaxf(wy, __shfl_xor(wy, o, 64));
    nb_before = __shfl(wy, 0, 64);
    nb_after = __shfl(wy, 8, 64);
  }
  if (it.len == 64 * K && (((uintptr_t)src) & 15u) == 0) {
    // full, 16-byte aligned tile (the common case): no per-element tests
    const float4 *src4 = reinterpret_cast<const float4 *>(__builtin_assume_aligned(src, 16));
#pragma unroll
    for (int r = 0; r < NV; ++r) v[r] = src4[lane + 64 * r];
    bool range_ok = true;
    float frac = 0.0f;  // sum of fractions of coordinate * 2^30: 0 iff all on grid
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int e = 2 * (lane + 64 * r);
      if (validate) {
        range_ok = range_ok && __builtin_fabsf(v[r].x - 0.5f) <= 0.5f &&
                   __builtin_fabsf(v[r].z - 0.5f) <= 0.5f && __builtin_fabsf(v[r].y) <= 1.0f &&
                   __builtin_fabsf(v[r].w) <= 1.0f;
        frac += (__builtin_amdgcn_fractf(v[r].x * 0x1p30f) +
                 __builtin_amdgcn_fractf(v[r].y * 0x1p30f)) +
                (__builtin_amdgcn_fractf(v[r].z * 0x1p30f) +
                 __builtin_amdgcn_fractf(v[r].w * 0x1p30f));
      }
      float4 *d = reinterpret_cast<float4 *>(
          __builtin_assume_aligned(sxy + (e / K) * S + (e % K), 16));
      *d = v[r];
    }
    if (!range_ok) err = UH_ERR_RANGE;
    else if (frac != 0.0f) err = UH_ERR_GRID;
  } else {
    const bool al = (((uintptr_t)src) & 15u) == 0;
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int e = 2 * (lane + 64 * r);
      if (e + 1 < it.len) {
        if (al) {
          v[r] = *reinterpret_cast<const float4 *>(src + e);
        } else {
          const float2 a = src[e], b = src[e + 1];
          v[r] = make_float4(a.x, a.y, b.x, b.y);
        }
      } else if (e < it.len) {
        const float2 a = src[e];
        v[r] = make_float4(a.x, a.y, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int e = 2 * (lane + 64 * r);
      if (e < it.len) {
        float2 *d = sxy + (e / K) * S + (e % K);
        if (validate) {
          err = min(err, check_point(make_float2(v[r].x, v[r].y)));
          if (e + 1 < it.len) err = min(err, check_point(make_float2(v[r].z, v[r].w)));
        }
        if (e + 1 < it.len)
          *reinterpret_cast<float4 *>(d) = v[r];
        else
          *d = make_float2(v[r].x, v[r].y);
      }
    }
  }
  wave_sync();
  const int my_len = min(max(it.len - lane * K, 0), K);
  float2 *st = sxy + lane * S;
  uint16_t *sl = sid + lane * S;
  float2 p[K];
#pragma unroll
  for (int k = 0; k < K / 2; ++k) {
    const float4 q = *reinterpret_cast<const float4 *>(st + 2 * k);
    p[2 * k] = make_float2(q.x, q.y);
    p[2 * k + 1] = make_float2(q.z, q.w);
  }

  // ---- 2. strip pass 1
  OrientCount oc;
  float ymax = -2.0f;  // below every valid y
  {
    float px = __shfl_up(p[K - 1].x, 1, 64);  // last point of the previous strip
    if (lane == 0) px = prev_tile_x;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (i < my_len) {
        ymax = fmaxf(ymax, p[i].y);
        if (validate && p[i].x < px) err = min(err, UH_ERR_UNSORTED);
        px = p[i].x;
      }
    }
  }
  const float incp = wave_prefix_max(ymax), incs = wave_suffix_max(ymax);
  float exp_pre = __shfl_up(incp, 1, 64), exp_suf = __shfl_down(incs, 1, 64);
  if (lane == 0) exp_pre = -2.0f;
  if (lane == 63) exp_suf = -2.0f;
  exp_pre = fmaxf(exp_pre, nb_before);
  exp_suf = fmaxf(exp_suf, nb_after);

  // ---- 3. strip pass 2: elimination (from registers)
  uint32_t keep = 0;
  {
    float bm = exp_pre;  // max y over earlier points of the tile
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (i < my_len && (p[i].y > bm || p[i].y >= exp_suf)) keep |= 1u << i;
      bm = fmaxf(bm, p[i].y);
    }
  }
  // Survivors of the whole wave, counted and ranked by a wave prefix sum.
  const int nk = __builtin_popcount(keep);
  int koff = nk;  // inclusive prefix sum of nk over the lanes
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(koff, o, 64);
    if (lane >= o) koff += y;
  }
  const int nsurv = __shfl(koff, 63, 64);
  koff -= nk;
  int nleaf;
  if (!it.final_ && nsurv <= TILE_LIST_MAX) {
    // Few survivors: hand them on, in order, as a point list; the merge
    // kernel turns them into a hood after eliminating across many tiles.
    err = wave_min(err);
    const int rel0 = (int)(it.start - sstart);
    int r = koff;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if ((keep >> i) & 1u) {
        A.ws_xy[it.start + r] = p[i];
        A.ws_idx[it.start + r] = rel0 + lane * K + i;
        ++r;
      }
    }
    if (lane == 0) {
      cnt_out[blockIdx.x] = (int)((uint32_t)nsurv | POINTS_FLAG);
      if (err) atomicMin(&A.set_status[it.set], err);
    }
    flush_wave_stats(A, it.set, oc);
    return;
  } else {
    // Many survivors: the serial strip hood over each strip's survivors
    // (re-read from LDS; the stack overwrites the slot from its start,
    // never past a survivor still to be read), then the non-empty strip
    // hoods are the leaves.
    int cnt = 0;
    float2 t1 = make_float2(0.f, 0.f), t2 = t1;  // stack top, second
    while (keep) {
      const int i = __builtin_ctz(keep);
      keep &= keep - 1;
      const float2 r = st[i];
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
    // Leaves of the merge tree: the non-empty strip hoods, in order.
    // Nothing between two consecutive leaves survived, so merging
    // neighbouring leaves is merging hoods of x-adjacent point sets.
    const uint64_t ne = __ballot(cnt > 0);
    nleaf = __builtin_popcountll(ne);
    if (cnt > 0) sblk[__builtin_popcountll(ne & ((1ull << lane) - 1ull))] = make_int2(lane * S, cnt);
    wave_sync();
  }

  // ---- 4. rounds of Wagener merges over the leaves
  wave_rounds(sxy, sid, sblk, nleaf, oc, fe);

  // ---- 5. output
  err = wave_min(err);
  const int hb = nleaf ? sblk[0].x : 0, hc = nleaf ? sblk[0].y : 0;
  const int rel0 = (int)(it.start - sstart);
  if (it.final_) {
    int32_t *dst = A.out_idx + sstart;
    for (int k = lane; k < hc; k += 64) dst[k] = rel0 + (int)sid[hb + k];
    if (lane == 0) A.out_counts[it.set] = err ? err : hc;
  } else {
    for (int k = lane; k < hc; k += 64) {
      A.ws_xy[it.start + k] = sxy[hb + k];
      A.ws_idx[it.start + k] = rel0 + (int)sid[hb + k];
    }
    if (lane == 0) {
      cnt_out[blockIdx.x] = hc;
      if (err) atomicMin(&A.set_status[it.set], err);
    }
  }
  flush_wave_stats(A, it.set, oc);
}

// ---------------------------------------------------------------- merges
// Exclusive prefix sum of one value per thread over the workgroup.
__device__ __forceinline__ int block_exclusive_scan(int v, int *swave, int &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) swave[w] = x;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int k = 0; k < BLOCK / 64; ++k) {
    if (k < w) before += swave[k];
    total += swave[k];
  }
  return before + x - v;
}

// One workgroup merges the hoods of up to F = 256 consecutive blocks of the
// previous level of one set (log2 F more rounds).  When their corners fit
// in LDS: gather them back to back, six rounds inside each wave (64
// children -> 1), then wave 0 merges the four wave hoods.  Otherwise the
// same rounds run in place in the workspace (global memory), each merge by
// a group of lanes with workgroup barriers between the reads and writes of
// the compaction.
__global__ __launch_bounds__(BLOCK) void merge_kernel(
    RunArgs A, const MergeItem *items, const int64_t *child_off,
    const int32_t *child_cnt, int32_t *cnt_out) {
  __shared__ float2 bxy[VMAX];
  __shared__ int32_t bid[VMAX];
  __shared__ int bcnt[BLOCK];
  __shared__ int2 sblk[BLOCK];  // LDS path: (base, count) per child block
  __shared__ int2 sres[BLOCK / 2];
  __shared__ int swave[BLOCK / 64];
  __shared__ int smax;

  const MergeItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const bool fe = (A.flags & UH_FLAG_FORCE_FALLBACK) != 0;
  const int nch = it.nch;

  // a child is a hood, or (POINTS_FLAG) a tile's sorted surviving points
  const uint32_t craw = tid < nch ? (uint32_t)child_cnt[it.child0 + tid] : 0u;
  const bool pts = (craw & POINTS_FLAG) != 0;
  const int c = (int)(craw & ~POINTS_FLAG);
  int V;
  const int o = block_exclusive_scan(c, swave, V);
  bcnt[tid] = c;
  int npow = 1;
  while (npow < nch) npow <<= 1;
  OrientCount oc;
  __syncthreads();

  if (V <= VMAX) {
    // ---- gather: thread k copies child k's corners (independent loads)
    if (tid < nch) {
      const int64_t g = child_off[it.child0 + tid];
      for (int e = 0; e < c; ++e) {
        bxy[o + e] = A.ws_xy[g + e];
        bid[o + e] = A.ws_idx[g + e];
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
      float cmax = -2.0f;
      for (int e = 0; e < c; ++e) cmax = fmaxf(cmax, bxy[o + e].y);
      const float incp = wave_prefix_max(cmax), incs = wave_suffix_max(cmax);
      __shared__ float swp[BLOCK / 64], sws[BLOCK / 64];
      if (lane == 63) swp[w] = incp;
      if (lane == 0) sws[w] = incs;
      float pre = __shfl_up(incp, 1, 64), suf = __shfl_down(incs, 1, 64);
      if (lane == 0) pre = -2.0f;
      if (lane == 63) suf = -2.0f;
      __syncthreads();
      for (int k = 0; k < BLOCK / 64; ++k) {
        if (k < w) pre = fmaxf(pre, swp[k]);
        if (k > w) suf = fmaxf(suf, sws[k]);
      }
      int kept = 0;
      for (int e = 0; e < c; ++e) {
        const float2 q = bxy[o + e];
        const bool keep = q.y > pre || q.y >= suf;
        pre = fmaxf(pre, q.y);
        if (keep) {
          const int32_t qi = bid[o + e];
          bxy[o + kept] = q;
          bid[o + kept] = qi;
          ++kept;
        }
      }
      // a point-list child becomes a hood: the serial strip hood of its
      // surviving points (the paper's serial hoods of small strips)
      if (pts && kept > 0) kept = chain_inplace(bxy + o, bid + o, kept, oc, fe);
      // leaves: the non-empty children, in order, 64 per wave
      const uint64_t ne = __ballot(kept > 0);
      if (kept > 0)
        sblk[(w << 6) + __builtin_popcountll(ne & ((1ull << lane) - 1ull))] = make_int2(o, kept);
      if (lane == 0) swave[w] = __builtin_popcountll(ne);
    }
    __syncthreads();
    wave_rounds(bxy, bid, sblk + (w << 6), swave[w], oc, fe);
    __syncthreads();
    if (w == 0) {
      // the wave hoods (one per wave that had leaves), left to right
      int nb0 = 0, nc0 = 0;
      bool have = false;
      for (int k = 0; k < BLOCK / 64; ++k) {
        if (swave[k] == 0) continue;
        const int2 Q = sblk[k << 6];
        if (!have) {
          nb0 = Q.x;
          nc0 = Q.y;
          have = true;
          continue;
        }
        int nb, nc;
        merge_blocks(bxy, bid, nb0, nc0, Q.x, Q.y, 6, lane, 0, nb, nc, oc, fe);
        wave_sync();
        nb0 = nb;
        nc0 = nc;
      }
      if (lane == 0) sblk[0] = make_int2(nb0, nc0);
      wave_sync();
      const int hb = sblk[0].x, hc = sblk[0].y;
      if (it.final_) {
        int32_t *dst = A.out_idx + A.set_start[it.set];
        for (int k = lane; k < hc; k += 64) dst[k] = bid[hb + k];
        if (lane == 0) {
          const int st = A.set_status[it.set];
          A.out_counts[it.set] = st ? st : hc;
        }
      } else {
        for (int k = lane; k < hc; k += 64) {
          A.ws_xy[it.off + k] = bxy[hb + k];
          A.ws_idx[it.off + k] = bid[hb + k];
        }
        if (lane == 0) cnt_out[blockIdx.x] = hc;
      }
    }
    flush_wave_stats(A, it.set, oc);
    return;
  }

  // ---- too large for LDS: the same rounds in place in the workspace
  if (pts && c > 0) {  // point-list children first become hoods, in place
    const int64_t g = child_off[it.child0 + tid];
    bcnt[tid] = chain_inplace(A.ws_xy + g, A.ws_idx + g, c, oc, fe);
  }
  __syncthreads();
#pragma unroll 1
  for (int j = 0; (1 << j) < nch; ++j) {
    const int M = npow >> (j + 1);
    const int G = BLOCK / M;
    const int m = tid / G, t = tid % G;
    const int lp = (2 * m) << j, lq = (2 * m + 1) << j;
    int a = -1, b = 0, hp = 0, hqe = 0, qs = 0;
    float2 *P = nullptr, *Q = nullptr;
    int32_t *Pid = nullptr, *Qid = nullptr;
    if (tid == 0) smax = 0;
    if (lp < nch && lq < nch) {
      const int64_t op = child_off[it.child0 + lp], oq = child_off[it.child0 + lq];
      P = A.ws_xy + op;
      Q = A.ws_xy + oq;
      Pid = A.ws_idx + op;
      Qid = A.ws_idx + oq;
      hp = bcnt[lp];
      const int hq = bcnt[lq];
      if (hp > 0 && hq > 0) junction_rule(P[hp - 1], Q[0], hp, qs);
      hqe = hq - qs;
      a = hp - 1;
      const int L = G < 64 ? G : 64;
      if (hp > 0 && hqe > 0 && t < L)
        bridge_search<const float2 *>(P, hp, Q + qs, hqe, L, t, (tid & 63) - t, a, b, oc,
                                      fe);
    }
    __syncthreads();  // smax cleared, and searches done reading
    if (G > 64) {
      if (t == 0) sres[m] = make_int2(a, b);
      __syncthreads();
      const int2 rr = sres[m];
      a = rr.x;
      b = rr.y;
    }
    const bool active = lp < nch && lq < nch;
    const int nsurv = active ? hqe - b : 0;
    const int chunks = (nsurv + G - 1) / G;
    if (t == 0 && active) atomicMax(&smax, chunks);
    __syncthreads();
    const int maxchunks = smax;
    // left shift Q[b..] to P[a+1..]: destination never passes the source,
    // so reading chunk c before anyone writes it keeps every value intact
    for (int ch = 0; ch < maxchunks; ++ch) {
      const int e = ch * G + t;
      float2 v = make_float2(0.f, 0.f);
      int32_t vi = 0;
      const bool mine = e < nsurv;
      if (mine) {
        v = Q[qs + b + e];
        vi = Qid[qs + b + e];
      }
      __syncthreads();
      if (mine) {
        P[a + 1 + e] = v;
        Pid[a + 1 + e] = vi;
      }
      __syncthreads();
    }
    if (t == 0 && active) bcnt[lp] = a + 1 + nsurv;
    __syncthreads();
  }
  const int hc = bcnt[0];
  const float2 *res_xy = A.ws_xy + it.off;
  const int32_t *res_id = A.ws_idx + it.off;
  if (it.final_) {
    int32_t *dst = A.out_idx + A.set_start[it.set];
    for (int k = tid; k < hc; k += BLOCK) dst[k] = res_id[k];
    if (tid == 0) {
      const int st = A.set_status[it.set];
      A.out_counts[it.set] = st ? st : hc;
    }
  } else {
    (void)res_xy;
    if (tid == 0) cnt_out[blockIdx.x] = hc;
  }
  flush_wave_stats(A, it.set, oc);
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

struct upper_hull_plan {
  int device = 0;
  int32_t S = 0;
  int64_t N = 0;
  int K = 16, T = 4096, F = 256;
  uint32_t flags = 0;
  int32_t ntiles = 0;
  std::vector<int32_t> pass_items;  // merge items per pass
  // device memory
  int64_t *d_set_start = nullptr;
  TileItem *d_tiles = nullptr;
  int64_t *d_tile_off = nullptr;
  int32_t *d_cnt0 = nullptr;
  std::vector<MergeItem *> d_items;
  std::vector<int64_t *> d_off;   // per pass: item slot offsets
  std::vector<int32_t *> d_cnt;   // per pass: item corner counts
  float2 *ws_xy = nullptr;
  int32_t *ws_idx = nullptr;
  int32_t *set_status = nullptr;
  // graph cache: (points, out_idx, out_counts, stats) -> exec
  std::map<std::tuple<const void *, void *, void *, void *>, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;
  hipEvent_t probe_before = nullptr, probe_after = nullptr;
  std::mutex mu;
};

namespace {

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

void free_plan_memory(upper_hull_plan *p) {
  hipFree(p->d_set_start);
  hipFree(p->d_tiles);
  hipFree(p->d_tile_off);
  hipFree(p->d_cnt0);
  for (auto *q : p->d_items) hipFree(q);
  for (auto *q : p->d_off) hipFree(q);
  for (auto *q : p->d_cnt) hipFree(q);
  hipFree(p->ws_xy);
  hipFree(p->ws_idx);
  hipFree(p->set_status);
  for (auto &kv : p->graphs) hipGraphExecDestroy(kv.second);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
}

int enqueue_run(upper_hull_plan *p, const RunArgs &A, hipStream_t stream) {
  {
    const int nb = (p->S + 255) / 256;
    hipLaunchKernelGGL(init_kernel, dim3(nb), dim3(256), 0, stream, p->S, A);
  }
  if (p->ntiles > 0) {
    const dim3 grid(p->ntiles), blk(64);
    if (p->probe_before && hipEventRecord(p->probe_before, stream) != hipSuccess)
      return UH_ERR_HIP;
    switch (p->K) {
      case 4: hipLaunchKernelGGL(tile_kernel<4>, grid, blk, 0, stream, A, p->d_tiles, p->d_cnt0); break;
      case 8: hipLaunchKernelGGL(tile_kernel<8>, grid, blk, 0, stream, A, p->d_tiles, p->d_cnt0); break;
      case 16: hipLaunchKernelGGL(tile_kernel<16>, grid, blk, 0, stream, A, p->d_tiles, p->d_cnt0); break;
      case 32: hipLaunchKernelGGL(tile_kernel<32>, grid, blk, 0, stream, A, p->d_tiles, p->d_cnt0); break;
      default: return UH_ERR_ARG;
    }
    if (p->probe_after && hipEventRecord(p->probe_after, stream) != hipSuccess)
      return UH_ERR_HIP;
  }
  for (size_t ps = 0; ps < p->pass_items.size(); ++ps) {
    const int64_t *coff = ps == 0 ? p->d_tile_off : p->d_off[ps - 1];
    const int32_t *ccnt = ps == 0 ? p->d_cnt0 : p->d_cnt[ps - 1];
    hipLaunchKernelGGL(merge_kernel, dim3(p->pass_items[ps]), dim3(BLOCK), 0, stream, A,
                       p->d_items[ps], coff, ccnt, p->d_cnt[ps]);
  }
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

std::mutex g_cache_mu;
std::map<std::pair<int, int64_t>, upper_hull_plan *> g_single_plans;

}  // namespace

extern "C" {

const char *upper_hull_status_string(int status) {
  switch (status) {
    case UH_OK: return "ok";
    case UH_ERR_ARG: return "invalid argument";
    case UH_ERR_ALLOC: return "device allocation failed";
    case UH_ERR_HIP: return "HIP runtime error";
    case UH_ERR_CAPTURE: return "plan creation not allowed during stream capture";
    case UH_ERR_UNSORTED: return "data error: x not non-decreasing";
    case UH_ERR_RANGE: return "data error: coordinate out of range or not finite";
    case UH_ERR_GRID: return "data error: coordinate not on the 2^-30 grid";
    default: return status >= 0 ? "ok (count)" : "unknown status";
  }
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
  int K = 16, F = 256;
  uint32_t flags = 0;
  if (config) {
    if (config->strip) K = config->strip;
    if (config->fan_in) F = config->fan_in;
    flags = config->flags;
  }
  if (K != 4 && K != 8 && K != 16 && K != 32) return UH_ERR_ARG;
  if (F < 2 || F > BLOCK || (F & (F - 1))) return UH_ERR_ARG;

  auto *p = new upper_hull_plan();
  hipGetDevice(&p->device);
  p->S = num_sets;
  p->N = set_offsets[num_sets];
  p->K = K;
  p->T = 64 * K;
  p->F = F;
  p->flags = flags;

  // level 0: tiles; then merge passes of fan-in F until one hood per set
  std::vector<TileItem> tiles;
  std::vector<int64_t> tile_off;
  std::vector<int32_t> first(num_sets), count(num_sets);  // blocks per set
  for (int32_t s = 0; s < num_sets; ++s) {
    const int64_t n = set_offsets[s + 1] - set_offsets[s];
    const int64_t nt = (n + p->T - 1) / p->T;
    first[s] = (int32_t)tiles.size();
    count[s] = (int32_t)nt;
    for (int64_t t = 0; t < nt; ++t) {
      TileItem it;
      it.start = set_offsets[s] + t * p->T;
      it.len = (int32_t)std::min<int64_t>(p->T, n - t * p->T);
      it.set = s;
      it.final_ = nt == 1;
      it.pad = 0;
      tiles.push_back(it);
      tile_off.push_back(it.start);
    }
  }
  p->ntiles = (int32_t)tiles.size();
  std::vector<int64_t> prev_off = tile_off;
  std::vector<std::vector<MergeItem>> passes;
  for (;;) {
    std::vector<MergeItem> items;
    std::vector<int32_t> nfirst(num_sets), ncount(num_sets);
    for (int32_t s = 0; s < num_sets; ++s) {
      nfirst[s] = (int32_t)items.size();
      ncount[s] = 0;
      if (count[s] <= 1) continue;
      const int32_t nitems = (count[s] + F - 1) / F;
      for (int32_t i = 0; i < nitems; ++i) {
        MergeItem m;
        m.child0 = first[s] + i * F;
        m.nch = std::min(F, count[s] - i * F);
        m.off = prev_off[m.child0];
        m.set = s;
        m.final_ = nitems == 1;
        items.push_back(m);
      }
      ncount[s] = nitems;
    }
    if (items.empty()) break;
    std::vector<int64_t> off(items.size());
    for (size_t i = 0; i < items.size(); ++i) off[i] = items[i].off;
    passes.push_back(items);
    prev_off = off;
    first = nfirst;
    // sets finished in this pass keep count 1 -> no further items
    for (int32_t s = 0; s < num_sets; ++s) count[s] = ncount[s];
  }

  int rc = UH_OK;
  std::vector<int64_t> so(set_offsets, set_offsets + num_sets + 1);
  rc = rc ? rc : dalloc(&p->d_set_start, so.size());
  rc = rc ? rc : upload(p->d_set_start, so);
  rc = rc ? rc : dalloc(&p->d_tiles, tiles.size());
  rc = rc ? rc : upload(p->d_tiles, tiles);
  rc = rc ? rc : dalloc(&p->d_tile_off, tile_off.size());
  rc = rc ? rc : upload(p->d_tile_off, tile_off);
  rc = rc ? rc : dalloc(&p->d_cnt0, tiles.size());
  for (auto &items : passes) {
    if (rc) break;
    MergeItem *di = nullptr;
    int64_t *doff = nullptr;
    int32_t *dcnt = nullptr;
    std::vector<int64_t> off(items.size());
    for (size_t i = 0; i < items.size(); ++i) off[i] = items[i].off;
    rc = rc ? rc : dalloc(&di, items.size());
    rc = rc ? rc : upload(di, items);
    rc = rc ? rc : dalloc(&doff, items.size());
    rc = rc ? rc : upload(doff, off);
    rc = rc ? rc : dalloc(&dcnt, items.size());
    p->d_items.push_back(di);
    p->d_off.push_back(doff);
    p->d_cnt.push_back(dcnt);
    p->pass_items.push_back((int32_t)items.size());
  }
  rc = rc ? rc : dalloc(&p->ws_xy, (size_t)p->N);
  rc = rc ? rc : dalloc(&p->ws_idx, (size_t)p->N);
  rc = rc ? rc : dalloc(&p->set_status, (size_t)num_sets);
  if (rc) {
    free_plan_memory(p);
    delete p;
    return rc;
  }
  *out_plan = p;
  return UH_OK;
}

int upper_hull_plan_launches(const upper_hull_plan *plan) {
  if (!plan) return UH_ERR_ARG;
  return 1 + (plan->ntiles > 0) + (int)plan->pass_items.size();
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
  A.flags = p->flags;
  if (!(p->flags & UH_FLAG_GRAPH)) return enqueue_run(p, A, stream);

  std::lock_guard<std::mutex> lock(p->mu);
  auto key = std::make_tuple((const void *)points, (void *)out_idx, (void *)out_counts,
                             (void *)stats);
  auto itg = p->graphs.find(key);
  if (itg == p->graphs.end()) {
    if (!p->cap_stream &&
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return UH_ERR_HIP;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
      return UH_ERR_HIP;
    const int rc = enqueue_run(p, A, p->cap_stream);
    if (hipStreamEndCapture(p->cap_stream, &g) != hipSuccess || rc) {
      if (g) hipGraphDestroy(g);
      return rc ? rc : UH_ERR_HIP;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ie != hipSuccess) return UH_ERR_HIP;
    itg = p->graphs.emplace(key, ex).first;
  }
  return hipGraphLaunch(itg->second, stream) == hipSuccess ? UH_OK : UH_ERR_HIP;
}

void upper_hull_plan_destroy(upper_hull_plan *plan) {
  if (!plan) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(plan->device);
  hipDeviceSynchronize();
  free_plan_memory(plan);
  hipSetDevice(cur);
  delete plan;
}

int upper_hull(const float *points, int64_t n, int32_t *out_idx, int32_t *out_count,
               hipStream_t stream) {
  if (n < 0 || n > INT32_MAX || !out_count || (n > 0 && (!points || !out_idx)))
    return UH_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UH_ERR_HIP;
  upper_hull_plan *p = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto key = std::make_pair(dev, n);
    auto it = g_single_plans.find(key);
    if (it != g_single_plans.end()) {
      p = it->second;
    } else {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return UH_ERR_HIP;
      if (cs != hipStreamCaptureStatusNone) return UH_ERR_CAPTURE;
      if (g_single_plans.size() >= 8) {  // bounded cache: drop the oldest
        upper_hull_plan_destroy(g_single_plans.begin()->second);
        g_single_plans.erase(g_single_plans.begin());
      }
      const int64_t off[2] = {0, n};
      const int rc = upper_hull_plan_create(off, 1, nullptr, &p);
      if (rc) return rc;
      g_single_plans.emplace(key, p);
    }
  }
  return upper_hull_plan_run(p, points, out_idx, out_count, nullptr, stream);
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
