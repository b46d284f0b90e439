// radix_sort.hip -- the device sort by x in front of the hull for points in
// any order (declarations and the scheme in radix_sort.hpp).
#include "radix_sort.hpp"

#include <algorithm>
#include <vector>

#include "wagener_hull.h"

namespace uh_rs {
namespace {

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;  // scan entries per block

__device__ __forceinline__ uint32_t digit(uint32_t key, int shift) {
  return ((key & 0x7fffffffu) >> shift) & 0xffu;
}

// Lanes of the wave (among the valid ones) whose 8-bit digit equals this
// lane's.  Every lane of the wave must call it.
__device__ __forceinline__ uint64_t match8(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix sum of one value per thread over a workgroup of
// SC_THREADS threads; *total receives the sum.  ws: SC_THREADS / 64 slots.
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *ws, uint32_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[w] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < SC_THREADS / 64; ++k) {
    before += k < w ? ws[k] : 0u;
    all += ws[k];
  }
  __syncthreads();  // ws may be reused
  *total = all;
  return before + x - v;
}

// Per-block digit counts: hist[hist0 + d * nb] = keys of digit d in the block.
__global__ __launch_bounds__(RS_THREADS) void rs_upsweep(const RadixItem *items,
                                                         const float2 *pts,
                                                         const uint32_t *keys, int shift,
                                                         uint32_t *hist) {
  __shared__ uint32_t cnt[RS_BINS];
  const RadixItem it = items[blockIdx.x];
  const int t = threadIdx.x, lane = t & 63;
  uint32_t k[RS_ITEMS];
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    const int e = u * RS_THREADS + t;
    k[u] = 0u;
    if (e < it.len) k[u] = keys ? keys[it.start + e] : __float_as_uint(pts[it.start + e].x);
  }
  cnt[t] = 0u;  // RS_THREADS == RS_BINS
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    const bool valid = u * RS_THREADS + t < it.len;
    const uint32_t d = digit(k[u], shift);
    const uint64_t m = match8(d, valid);
    if (valid && (m & lt) == 0ull) atomicAdd(&cnt[d], (uint32_t)__builtin_popcountll(m));
  }
  __syncthreads();
  hist[it.hist0 + (int64_t)t * it.nb] = cnt[t];
}

// Exclusive scan of a[0, L): block sums, then the sums, then each block.
__global__ __launch_bounds__(SC_THREADS) void rs_scan_reduce(const uint32_t *a, int64_t L,
                                                             uint32_t *part) {
  __shared__ uint32_t ws[SC_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  uint32_t s = 0;
#pragma unroll
  for (int u = 0; u < SC_ITEMS; ++u) {
    const int64_t e = base + (int64_t)u * SC_THREADS + threadIdx.x;
    s += e < L ? a[e] : 0u;
  }
  uint32_t total;
  block_excl_sum(s, ws, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void rs_scan_partials(uint32_t *part, int n) {
  __shared__ uint32_t ws[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int c = 0; c < n; c += 1024) {
    const int e = c + threadIdx.x;
    const uint32_t v = e < n ? part[e] : 0u;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int k = 0; k < 16; ++k) {
      before += k < w ? ws[k] : 0u;
      all += ws[k];
    }
    if (e < n) part[e] = carry + before + x - v;
    carry += all;
    __syncthreads();
  }
}

__global__ __launch_bounds__(SC_THREADS) void rs_scan_apply(uint32_t *a, int64_t L,
                                                            const uint32_t *part) {
  __shared__ uint32_t ws[SC_THREADS / 64];
  // thread t owns entries [t * SC_ITEMS, (t + 1) * SC_ITEMS) of the block
  const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  uint32_t v[SC_ITEMS], s = 0;
#pragma unroll
  for (int u = 0; u < SC_ITEMS; ++u) {
    v[u] = base + u < L ? a[base + u] : 0u;
    s += v[u];
  }
  uint32_t total;
  uint32_t run = part[blockIdx.x] + block_excl_sum(s, ws, &total);
#pragma unroll
  for (int u = 0; u < SC_ITEMS; ++u) {
    if (base + u < L) a[base + u] = run;
    run += v[u];
  }
}

// One stable counting-sort pass of a block by the digit at `shift`: ranks
// within the block (by wave, then item, then lane: the input order), then
// the keys go through LDS in output order and leave with coalesced stores.
// Pass 0 reads the points themselves; the last pass writes sorted points
// and the permutation.
__global__ __launch_bounds__(RS_THREADS) void rs_downsweep(
    const RadixItem *items, const float2 *pts, const uint32_t *ikey, const float *iy,
    const int32_t *iidx, int shift, const uint32_t *hist, uint32_t *okey, float *oy,
    int32_t *oidx, float2 *osorted, int32_t *operm, int64_t n) {
  __shared__ uint32_t s_key[RS_TILE];
  __shared__ float s_y[RS_TILE];
  __shared__ int32_t s_idx[RS_TILE];
  __shared__ uint32_t wcnt[RS_THREADS / 64][RS_BINS];
  __shared__ uint32_t dbase[RS_BINS], gbase[RS_BINS], ws[RS_THREADS / 64];
  const RadixItem it = items[blockIdx.x];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  constexpr int WSPAN = RS_ITEMS * 64;  // keys per wave
  uint32_t k[RS_ITEMS], rank[RS_ITEMS];
  float yv[RS_ITEMS];
  int32_t iv[RS_ITEMS];
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    const int e = w * WSPAN + u * 64 + lane;
    k[u] = 0u;
    yv[u] = 0.0f;
    iv[u] = 0;
    if (e < it.len) {
      if (pts) {
        const float2 q = pts[it.start + e];
        k[u] = __float_as_uint(q.x);
        yv[u] = q.y;
        iv[u] = it.rel0 + e;
      } else {
        k[u] = ikey[it.start + e];
        yv[u] = iy[it.start + e];
        iv[u] = iidx[it.start + e];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RS_THREADS / 64; ++q) wcnt[q][t] = 0u;
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    const bool valid = w * WSPAN + u * 64 + lane < it.len;
    const uint32_t d = digit(k[u], shift);
    const uint64_t m = match8(d, valid);
    const uint32_t before = valid ? wcnt[w][d] : 0u;
    rank[u] = before + (uint32_t)__builtin_popcountll(m & lt);
    wave_lds_order();  // every lane has read its counter
    if (valid && (m & lt) == 0ull) wcnt[w][d] = before + (uint32_t)__builtin_popcountll(m);
    wave_lds_order();
  }
  __syncthreads();
  {
    // digit t: totals over the waves, each wave's start within the digit,
    // the digit's start within the block and in the output
    uint32_t c[RS_THREADS / 64], tot = 0;
#pragma unroll
    for (int q = 0; q < RS_THREADS / 64; ++q) {
      c[q] = wcnt[q][t];
      wcnt[q][t] = tot;
      tot += c[q];
    }
    uint32_t all;
    dbase[t] = block_excl_sum(tot, ws, &all);
    gbase[t] = hist[it.hist0 + (int64_t)t * it.nb];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    if (w * WSPAN + u * 64 + lane < it.len) {
      const uint32_t d = digit(k[u], shift);
      const uint32_t pos = dbase[d] + wcnt[w][d] + rank[u];
      s_key[pos] = k[u];
      s_y[pos] = yv[u];
      s_idx[pos] = iv[u];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    const int i = u * RS_THREADS + t;
    if (i < it.len) {
      const uint32_t key = s_key[i];
      const uint32_t d = digit(key, shift);
      const int64_t g = (int64_t)gbase[d] + (i - (int64_t)dbase[d]);
      if (g < n) {  // always, by construction of the counts
        if (osorted) {
          osorted[g] = make_float2(__uint_as_float(key), s_y[i]);
          operm[g] = s_idx[i];
        } else {
          okey[g] = key;
          oy[g] = s_y[i];
          oidx[g] = s_idx[i];
        }
      }
    }
  }
}

template <class T>
int dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, count * sizeof(T)) == hipSuccess ? UH_OK : UH_ERR_ALLOC;
}

}  // namespace

int radix_plan_build(const int64_t *set_offsets, int32_t num_sets, RadixPlan *rp) {
  std::vector<RadixItem> items;
  for (int32_t s = 0; s < num_sets; ++s) {
    const int64_t n = set_offsets[s + 1] - set_offsets[s];
    const int32_t nb = (int32_t)((n + RS_TILE - 1) / RS_TILE);
    const int32_t b0 = (int32_t)items.size();
    for (int32_t b = 0; b < nb; ++b) {
      RadixItem it;
      it.start = set_offsets[s] + (int64_t)b * RS_TILE;
      it.len = (int32_t)std::min<int64_t>(RS_TILE, n - (int64_t)b * RS_TILE);
      it.rel0 = b * RS_TILE;
      it.hist0 = RS_BINS * b0 + b;
      it.nb = nb;
      items.push_back(it);
    }
  }
  const int64_t N = set_offsets[num_sets];
  rp->nblocks = (int32_t)items.size();
  rp->nhist = (int64_t)RS_BINS * rp->nblocks;
  rp->npart = (int32_t)((rp->nhist + SC_TILE - 1) / SC_TILE);
  int rc = dalloc(&rp->items, items.size());
  if (!rc && !items.empty() &&
      hipMemcpy(rp->items, items.data(), items.size() * sizeof(RadixItem),
                hipMemcpyHostToDevice) != hipSuccess)
    rc = UH_ERR_HIP;
  rc = rc ? rc : dalloc(&rp->hist, (size_t)rp->nhist);
  rc = rc ? rc : dalloc(&rp->part, (size_t)rp->npart);
  for (int b = 0; b < 2 && !rc; ++b) {
    rc = rc ? rc : dalloc(&rp->key[b], (size_t)N);
    rc = rc ? rc : dalloc(&rp->y[b], (size_t)N);
    rc = rc ? rc : dalloc(&rp->idx[b], (size_t)N);
  }
  return rc;
}

void radix_plan_free(RadixPlan *rp) {
  (void)hipFree(rp->items);
  (void)hipFree(rp->hist);
  (void)hipFree(rp->part);
  for (int b = 0; b < 2; ++b) {
    (void)hipFree(rp->key[b]);
    (void)hipFree(rp->y[b]);
    (void)hipFree(rp->idx[b]);
  }
  *rp = RadixPlan();
}

int radix_sort_enqueue(const RadixPlan &rp, const float2 *pts, int64_t n, float2 *sorted,
                       int32_t *perm, hipStream_t stream) {
  if (rp.nblocks == 0) return UH_OK;
  for (int pass = 0; pass < RS_PASSES; ++pass) {
    const int shift = 8 * pass;
    const bool first = pass == 0, last = pass == RS_PASSES - 1;
    const int in = (pass + 1) & 1, out = pass & 1;  // pass p writes buffer p & 1
    hipLaunchKernelGGL(rs_upsweep, dim3(rp.nblocks), dim3(RS_THREADS), 0, stream, rp.items,
                       first ? pts : nullptr, first ? nullptr : rp.key[in], shift, rp.hist);
    hipLaunchKernelGGL(rs_scan_reduce, dim3(rp.npart), dim3(SC_THREADS), 0, stream, rp.hist,
                       rp.nhist, rp.part);
    hipLaunchKernelGGL(rs_scan_partials, dim3(1), dim3(1024), 0, stream, rp.part, rp.npart);
    hipLaunchKernelGGL(rs_scan_apply, dim3(rp.npart), dim3(SC_THREADS), 0, stream, rp.hist,
                       rp.nhist, rp.part);
    hipLaunchKernelGGL(rs_downsweep, dim3(rp.nblocks), dim3(RS_THREADS), 0, stream, rp.items,
                       first ? pts : nullptr, first ? nullptr : rp.key[in],
                       first ? nullptr : rp.y[in], first ? nullptr : rp.idx[in], shift, rp.hist,
                       last ? nullptr : rp.key[out], last ? nullptr : rp.y[out],
                       last ? nullptr : rp.idx[out], last ? sorted : nullptr,
                       last ? perm : nullptr, n);
  }
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

}  // namespace uh_rs
