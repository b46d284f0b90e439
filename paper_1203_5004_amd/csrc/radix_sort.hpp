// radix_sort.hpp -- device sort of every set's points by x (stable), the
// front end for points given in any order.
//
// The method needs its points in left-to-right order (the problem statement
// of the paper's section on the CUDA version of Wagener's algorithm).  For
// other input the library sorts each set by x on the device, keeping equal x
// in input order, so every "lowest index" tie rule still refers to input
// indices; the hull indices are mapped back through the permutation.
//
// Least-significant-digit radix sort, five passes of 6 bits over the low 30
// float bits of x (for x in [0, 1] those order like the values, and -0.0
// sorts with +0.0; a value outside [0, 1] lands somewhere and is reported by
// the hull's checks).  Sets are sorted independently in one pass sequence:
// every block of up to RS_TILE points lies in one set, and a key's output
// position is its set's start, plus the keys of its set with a smaller
// digit, plus those with its digit in earlier blocks of the set, plus its
// rank in its block.  The per-block digit counts are summed over chunks of
// blocks, scanned over the chunks of each set, and rescanned inside each
// chunk, all with one lane per digit and coalesced rows.  Six-bit digits
// give runs of about 64 keys per digit and block; between passes a key
// travels with its payload as one 12-byte record, so the scattered stores of
// a pass write runs of about 768 bytes (separate key and payload arrays,
// which would let the count pass read 4 bytes a key, measured slower).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uh_rs {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;                      // keys per thread
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;    // keys per block
constexpr int RS_BITS = 6;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_PASSES = 5;
constexpr int RS_CHUNK = 256;  // blocks per chunk of the scan

struct RadixItem {   // one block of the sort: a range of one set
  int64_t start;     // first point (absolute)
  int32_t len;       // 1 .. RS_TILE
  int32_t rel0;      // start minus the set's start
};

struct RadixChunk {  // up to RS_CHUNK consecutive blocks of one set
  int32_t b0, nb;    // first block, blocks
  int32_t set;       // index among the non-empty sets
  int32_t pad;
};

struct RadixSet {    // a non-empty set
  int64_t start;     // its first point
  int32_t c0, nc;    // its chunks
};

struct RadixRec {    // a key and its payload between passes (12 bytes)
  uint32_t key;      // bits of x
  float y;
  int32_t idx;       // set-relative input index
};

struct RadixPlan {
  int32_t nblocks = 0, nchunks = 0, nsets = 0;
  RadixItem *items = nullptr;    // [nblocks]
  RadixChunk *chunks = nullptr;  // [nchunks]
  RadixSet *sets = nullptr;      // [nsets]
  uint32_t *hist = nullptr;      // [nblocks * RS_BINS] digit counts, then output starts
  uint32_t *csum = nullptr;      // [nchunks * RS_BINS] chunk sums, then chunk starts
  uint32_t *dbase = nullptr;     // [nsets * RS_BINS] where each digit of a set starts
  RadixRec *rec[2] = {nullptr, nullptr};  // records between passes (ping-pong)
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
