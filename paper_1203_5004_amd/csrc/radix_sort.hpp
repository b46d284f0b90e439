// radix_sort.hpp -- device sort of every set's points by x (stable), the
// front end for points given in any order.
//
// The method needs its points in left-to-right order (the problem statement
// of the paper's section on the CUDA version of Wagener's algorithm).  For
// other input the library sorts each set by x on the device, keeping equal x
// in input order, so every "lowest index" tie rule still refers to input
// indices; the hull indices are mapped back through the permutation.
//
// Least-significant-digit radix sort, four passes of 8 bits over the float
// bits of x with the sign bit cleared (for x in [0, 1] the bits order like
// the values; -0.0 sorts with +0.0).  Sets are sorted independently in one
// pass sequence: every block of up to RS_TILE points lies in one set, and the
// per-block digit counts are laid out set by set, digit-major within a set,
// so one exclusive scan over all of them gives every (set, digit, block) its
// absolute output position.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uh_rs {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;                      // keys per thread
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;    // keys per block
constexpr int RS_BINS = 256;
constexpr int RS_PASSES = 4;

struct RadixItem {   // one block of the sort: a range of one set
  int64_t start;     // first point (absolute)
  int32_t len;       // 1 .. RS_TILE
  int32_t rel0;      // start minus the set's start
  int32_t hist0;     // counts of digit d go to hist[hist0 + d * nb]
  int32_t nb;        // blocks of this set
};

struct RadixPlan {
  int32_t nblocks = 0;
  int64_t nhist = 0;             // RS_BINS * nblocks
  int32_t npart = 0;             // scan partials
  RadixItem *items = nullptr;    // [nblocks]
  uint32_t *hist = nullptr;      // [nhist]
  uint32_t *part = nullptr;      // [npart]
  uint32_t *key[2] = {nullptr, nullptr};  // x bits, per pass (ping-pong)
  float *y[2] = {nullptr, nullptr};
  int32_t *idx[2] = {nullptr, nullptr};   // set-relative input index
};

// Builds the blocks and allocates the buffers for sets set_offsets[0..S].
// Returns 0 or a negative status (UH_ERR_ALLOC).
int radix_plan_build(const int64_t *set_offsets, int32_t num_sets, RadixPlan *rp);
void radix_plan_free(RadixPlan *rp);

// Enqueues the sort of pts (n points) on stream: sorted[k] is the point at
// sorted position k, perm[k] its set-relative input index.
int radix_sort_enqueue(const RadixPlan &rp, const float2 *pts, int64_t n, float2 *sorted,
                       int32_t *perm, hipStream_t stream);

}  // namespace uh_rs
