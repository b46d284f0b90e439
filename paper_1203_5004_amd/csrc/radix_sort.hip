// radix_sort.hip -- the device sort by x in front of the hull for points in
// any order (declarations and the scheme in radix_sort.hpp).
#include "radix_sort.hpp"

#include <algorithm>
#include <vector>

#include "wagener_hull.h"

namespace uh_rs {
namespace {

static_assert(RS_BINS == 64, "the scan kernels run one lane per digit in one wave");
static_assert(RS_BITS * RS_PASSES == 30, "the passes cover the low 30 bits of x");
static_assert(RS_THREADS == 256 && RS_TILE == RS_THREADS * RS_ITEMS, "block shape");

__device__ __forceinline__ uint32_t digit(uint32_t key, int shift) {
  return (key >> shift) & (RS_BINS - 1);  // shift + RS_BITS <= 30: the sign bit never counts
}

// Lanes of the wave (among the valid ones) whose digit equals this lane's.
// Every lane of the wave must call it.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < RS_BITS; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Exclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_excl_sum(uint32_t v) {
  const int lane = threadIdx.x & 63;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x - v;
}

// Per-block digit counts: hist[b * RS_BINS + d].  Each wave counts into
// its own LDS row (plain LDS atomics; lanes of one digit queue on one bank).
__global__ __launch_bounds__(RS_THREADS) void rs_upsweep(const RadixItem *items,
                                                         const float2 *pts,
                                                         const RadixRec *rec, int shift,
                                                         uint32_t *hist) {
  __shared__ uint32_t cnt[RS_THREADS / 64][RS_BINS];
  const RadixItem it = items[blockIdx.x];
  const int t = threadIdx.x, w = t >> 6;
  uint32_t k[RS_ITEMS];
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    const int e = u * RS_THREADS + t;
    k[u] = 0u;
    if (e < it.len) k[u] = rec ? rec[it.start + e].key : __float_as_uint(pts[it.start + e].x);
  }
  if (t < RS_BINS) {
#pragma unroll
    for (int q = 0; q < RS_THREADS / 64; ++q) cnt[q][t] = 0u;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u)
    if (u * RS_THREADS + t < it.len) atomicAdd(&cnt[w][digit(k[u], shift)], 1u);
  __syncthreads();
  if (t < RS_BINS) {
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < RS_THREADS / 64; ++q) s += cnt[q][t];
    hist[(int64_t)blockIdx.x * RS_BINS + t] = s;
  }
}

// One wave per chunk, one lane per digit: the chunk's digit totals.
__global__ __launch_bounds__(64) void rs_chunk_sum(const RadixChunk *chunks,
                                                   const uint32_t *hist, uint32_t *csum) {
  const RadixChunk c = chunks[blockIdx.x];
  const int d = threadIdx.x;
  uint32_t s = 0;
  for (int b0 = 0; b0 < c.nb; b0 += 8) {  // eight loads in flight
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = b0 + j < c.nb ? hist[(int64_t)(c.b0 + b0 + j) * RS_BINS + d] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  csum[(int64_t)blockIdx.x * RS_BINS + d] = s;
}

// One wave per set: each chunk's start within its digit (in place), and
// where each digit of the set starts in the output.
__global__ __launch_bounds__(64) void rs_set_scan(const RadixSet *sets, uint32_t *csum,
                                                  uint32_t *dbase) {
  const RadixSet st = sets[blockIdx.x];
  const int d = threadIdx.x;
  uint32_t run = 0;
  for (int c0 = 0; c0 < st.nc; c0 += 8) {  // eight loads in flight, then the stores
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = c0 + j < st.nc ? csum[(int64_t)(st.c0 + c0 + j) * RS_BINS + d] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (c0 + j < st.nc) csum[(int64_t)(st.c0 + c0 + j) * RS_BINS + d] = run;
      run += v[j];
    }
  }
  dbase[(int64_t)blockIdx.x * RS_BINS + d] = (uint32_t)st.start + wave_excl_sum(run);
}

// One wave per chunk: every block's output start for each digit (in place).
__global__ __launch_bounds__(64) void rs_chunk_apply(const RadixChunk *chunks,
                                                     const uint32_t *csum,
                                                     const uint32_t *dbase, uint32_t *hist) {
  const RadixChunk c = chunks[blockIdx.x];
  const int d = threadIdx.x;
  uint32_t run = dbase[(int64_t)c.set * RS_BINS + d] + csum[(int64_t)blockIdx.x * RS_BINS + d];
  for (int b0 = 0; b0 < c.nb; b0 += 8) {  // eight loads in flight, then the stores
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = b0 + j < c.nb ? hist[(int64_t)(c.b0 + b0 + j) * RS_BINS + d] : 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (b0 + j < c.nb) hist[(int64_t)(c.b0 + b0 + j) * RS_BINS + d] = run;
      run += v[j];
    }
  }
}

// One stable counting-sort pass of a block by the digit at `shift`: ranks
// within the block (by wave, then item, then lane: the input order), then
// the keys go through LDS in output order and leave with coalesced stores.
// Pass 0 reads the points themselves; the last pass writes sorted points
// and the permutation.
__global__ __launch_bounds__(RS_THREADS) void rs_downsweep(
    const RadixItem *items, const float2 *pts, const RadixRec *irec, int shift,
    const uint32_t *hist, RadixRec *orec, float2 *osorted, int32_t *operm, int64_t n) {
  __shared__ uint32_t s_key[RS_TILE];
  __shared__ float s_y[RS_TILE];
  __shared__ int32_t s_idx[RS_TILE];
  __shared__ uint32_t wcnt[RS_THREADS / 64][RS_BINS];
  __shared__ uint32_t dstart[RS_BINS], gstart[RS_BINS];
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
        const RadixRec r = irec[it.start + e];
        k[u] = r.key;
        yv[u] = r.y;
        iv[u] = r.idx;
      }
    }
  }
  if (t < RS_BINS) {
#pragma unroll
    for (int q = 0; q < RS_THREADS / 64; ++q) wcnt[q][t] = 0u;
    gstart[t] = hist[(int64_t)blockIdx.x * RS_BINS + t];
  }
  __syncthreads();
  // Ranks within the wave: for each item, the lowest lane of every digit
  // adds the digit's count to the wave's counter and gets the count before
  // it (LDS atomics of one wave are done in issue order, so the items need
  // not wait for one another); the other lanes of the digit take it from
  // that lane.  Items go in groups of RS_GROUP, which bounds the registers
  // in flight.
  const uint64_t lt = (1ull << lane) - 1ull;
  constexpr int RS_GROUP = 4;
#pragma unroll
  for (int g = 0; g < RS_ITEMS; g += RS_GROUP) {
    uint32_t old[RS_GROUP];
    int lead[RS_GROUP];
#pragma unroll
    for (int j = 0; j < RS_GROUP; ++j) {
      const int u = g + j;
      const bool valid = w * WSPAN + u * 64 + lane < it.len;
      const uint32_t d = digit(k[u], shift);
      const uint64_t m = match_digit(d, valid);
      lead[j] = m ? __builtin_ctzll(m) : lane;
      rank[u] = (uint32_t)__builtin_popcountll(m & lt);
      old[j] = 0u;
      if (valid && (m & lt) == 0ull)
        old[j] = atomicAdd(&wcnt[w][d], (uint32_t)__builtin_popcountll(m));
    }
#pragma unroll
    for (int j = 0; j < RS_GROUP; ++j) rank[g + j] += (uint32_t)__shfl((int)old[j], lead[j], 64);
  }
  __syncthreads();
  if (t < RS_BINS) {
    // digit t: each wave's start within the digit, the digit's start in the block
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < RS_THREADS / 64; ++q) {
      const uint32_t c = wcnt[q][t];
      wcnt[q][t] = tot;
      tot += c;
    }
    dstart[t] = wave_excl_sum(tot);  // RS_BINS == 64: one wave holds every digit
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) {
    if (w * WSPAN + u * 64 + lane < it.len) {
      const uint32_t d = digit(k[u], shift);
      const uint32_t pos = dstart[d] + wcnt[w][d] + rank[u];
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
      const int64_t g = (int64_t)gstart[d] + (i - (int64_t)dstart[d]);
      if (g < n) {  // always, by construction of the counts
        if (osorted) {
          osorted[g] = make_float2(__uint_as_float(key), s_y[i]);
          operm[g] = s_idx[i];
        } else {
          RadixRec r;
          r.key = key;
          r.y = s_y[i];
          r.idx = s_idx[i];
          orec[g] = r;
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
  std::vector<RadixChunk> chunks;
  std::vector<RadixSet> sets;
  for (int32_t s = 0; s < num_sets; ++s) {
    const int64_t n = set_offsets[s + 1] - set_offsets[s];
    if (n == 0) continue;
    const int32_t nb = (int32_t)((n + RS_TILE - 1) / RS_TILE);
    const int32_t b0 = (int32_t)items.size();
    RadixSet st;
    st.start = set_offsets[s];
    st.c0 = (int32_t)chunks.size();
    st.nc = (nb + RS_CHUNK - 1) / RS_CHUNK;
    for (int32_t c = 0; c < st.nc; ++c) {
      RadixChunk ch;
      ch.b0 = b0 + c * RS_CHUNK;
      ch.nb = std::min(RS_CHUNK, nb - c * RS_CHUNK);
      ch.set = (int32_t)sets.size();
      ch.pad = 0;
      chunks.push_back(ch);
    }
    sets.push_back(st);
    for (int32_t b = 0; b < nb; ++b) {
      RadixItem it;
      it.start = set_offsets[s] + (int64_t)b * RS_TILE;
      it.len = (int32_t)std::min<int64_t>(RS_TILE, n - (int64_t)b * RS_TILE);
      it.rel0 = b * RS_TILE;
      items.push_back(it);
    }
  }
  const int64_t N = set_offsets[num_sets];
  rp->nblocks = (int32_t)items.size();
  rp->nchunks = (int32_t)chunks.size();
  rp->nsets = (int32_t)sets.size();
  int rc = dalloc(&rp->items, items.size());
  rc = rc ? rc : dalloc(&rp->chunks, chunks.size());
  rc = rc ? rc : dalloc(&rp->sets, sets.size());
  if (!rc && !items.empty() &&
      (hipMemcpy(rp->items, items.data(), items.size() * sizeof(RadixItem),
                 hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(rp->chunks, chunks.data(), chunks.size() * sizeof(RadixChunk),
                 hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(rp->sets, sets.data(), sets.size() * sizeof(RadixSet),
                 hipMemcpyHostToDevice) != hipSuccess))
    rc = UH_ERR_HIP;
  rc = rc ? rc : dalloc(&rp->hist, (size_t)rp->nblocks * RS_BINS);
  rc = rc ? rc : dalloc(&rp->csum, (size_t)rp->nchunks * RS_BINS);
  rc = rc ? rc : dalloc(&rp->dbase, (size_t)rp->nsets * RS_BINS);
  for (int b = 0; b < 2 && !rc; ++b) rc = dalloc(&rp->rec[b], (size_t)N);
  return rc;
}

void radix_plan_free(RadixPlan *rp) {
  (void)hipFree(rp->items);
  (void)hipFree(rp->chunks);
  (void)hipFree(rp->sets);
  (void)hipFree(rp->hist);
  (void)hipFree(rp->csum);
  (void)hipFree(rp->dbase);
  for (int b = 0; b < 2; ++b) (void)hipFree(rp->rec[b]);
  *rp = RadixPlan();
}

int radix_sort_enqueue(const RadixPlan &rp, const float2 *pts, int64_t n, float2 *sorted,
                       int32_t *perm, hipStream_t stream) {
  if (rp.nblocks == 0) return UH_OK;
  for (int pass = 0; pass < RS_PASSES; ++pass) {
    const int shift = RS_BITS * pass;
    const bool first = pass == 0, last = pass == RS_PASSES - 1;
    const int in = (pass + 1) & 1, out = pass & 1;  // pass p writes buffer p & 1
    hipLaunchKernelGGL(rs_upsweep, dim3(rp.nblocks), dim3(RS_THREADS), 0, stream, rp.items,
                       first ? pts : nullptr, first ? nullptr : rp.rec[in], shift, rp.hist);
    hipLaunchKernelGGL(rs_chunk_sum, dim3(rp.nchunks), dim3(64), 0, stream, rp.chunks, rp.hist,
                       rp.csum);
    hipLaunchKernelGGL(rs_set_scan, dim3(rp.nsets), dim3(64), 0, stream, rp.sets, rp.csum,
                       rp.dbase);
    hipLaunchKernelGGL(rs_chunk_apply, dim3(rp.nchunks), dim3(64), 0, stream, rp.chunks,
                       rp.csum, rp.dbase, rp.hist);
    hipLaunchKernelGGL(rs_downsweep, dim3(rp.nblocks), dim3(RS_THREADS), 0, stream, rp.items,
                       first ? pts : nullptr, first ? nullptr : rp.rec[in], shift, rp.hist,
                       last ? nullptr : rp.rec[out], last ? sorted : nullptr,
                       last ? perm : nullptr, n);
  }
  return hipGetLastError() == hipSuccess ? UH_OK : UH_ERR_HIP;
}

}  // namespace uh_rs
