/*
 * wagener_hull.h -- C ABI of the MI355X (gfx950) upper-hood / convex-hull
 * library.
 *
 * The library computes the upper hood (upper convex hull closed by downward
 * vertical rays) of x-sorted planar points with Wagener's merge, following
 * C. O Dunlaing, "CUDA implementation of Wagener's 2D convex hull PRAM
 * algorithm": adjacent blocks' hoods are joined pairwise, round after round,
 * each merge locating the common tangent (bridge) of the two hoods by a
 * sampled parallel search (the match-and-merge procedure, steps mam1-mam5)
 * and then keeping the left hood's corners up to the bridge and the right
 * hood's corners from it (mam6).  Everything runs on the device; the host is
 * touched only by the calls below.  On request the same read of the points
 * also gives the lower hood (UH_FLAG_BOTH_HOODS; convex_hull joins the two
 * into the 2-D convex hull the paper's title names), and points in any
 * order are first sorted by x on the device (UH_FLAG_UNSORTED).
 *
 * Conventions shared by every entry point
 *   - Points are float32 pairs (x, y), interleaved, i.e. the memory layout
 *     of HIP's float2; the pointer must be 8-byte aligned.
 *   - Contract on the data (the paper's problem statement, section
 *     "Wagener's algorithm, CUDA version", plus the readings below):
 *     x non-decreasing in input order (unless UH_FLAG_UNSORTED); x in
 *     [0, 1]; y in [-1, 1]; both
 *     coordinates multiples of 2^-30 (every float32 in [2^-7, 1] is).  On
 *     such data every orientation sign the library uses is exact.
 *   - Output: the corners of the strict upper hood as 0-based input indices
 *     (relative to the start of their set), strictly increasing, i.e. left
 *     to right.  Points inside a hood edge are not corners; at an x only the
 *     highest point can be a corner and identical points resolve to the
 *     lowest index.  Any n >= 0 is accepted (the paper asks for n a power of
 *     two); n = 0 gives no corner, n = 1 gives [0].
 *   - Device pointers are caller-owned; the library never frees them.
 *   - Calls are asynchronous on `stream` (0 = the null stream) and enqueue
 *     no host copy; results are valid once the stream has reached them.
 *   - Return value (synchronous): UH_OK, or a negative UH_ERR_* code for an
 *     argument, allocation or HIP-runtime problem; nothing is enqueued then.
 *   - Data errors (contract violations found while reading the points) are
 *     reported on the stream: the set's output count becomes the negative
 *     UH_ERR_UNSORTED / UH_ERR_RANGE / UH_ERR_GRID; its indices are then
 *     unspecified.
 *   - Thread safety: calls on different streams may run concurrently; one
 *     plan must not be run concurrently with itself (its workspace is
 *     shared by its runs).
 */
#ifndef WAGENER_HULL_H
#define WAGENER_HULL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define UH_OK 0
#define UH_ERR_ARG (-1)       /* NULL pointer, negative size, bad config   */
#define UH_ERR_ALLOC (-2)     /* device allocation failed                  */
#define UH_ERR_HIP (-3)       /* a HIP runtime call failed                 */
#define UH_ERR_CAPTURE (-4)   /* a plan would have to be built while the   */
                              /* stream is being captured into a graph     */
#define UH_ERR_UNSORTED (-10) /* data: x decreases somewhere               */
#define UH_ERR_RANGE (-11)    /* data: x outside [0,1], y outside [-1,1],  */
                              /*       or a NaN / infinity                 */
#define UH_ERR_GRID (-12)     /* data: a coordinate is not on the 2^-30    */
                              /*       grid                                */

/* Human-readable text of a status code (static storage, never NULL). */
const char *upper_hull_status_string(int status);

/* Per-set counters written by the batched entry point (device memory). */
typedef struct {
  uint64_t orient_evals; /* orientation tests evaluated                    */
  uint64_t fallbacks;    /* of which the FP32 filter could not decide and  */
                         /* the exact FP64 evaluation was used             */
} upper_hull_stats;

/* Plan options.  A NULL config pointer means the defaults. */
typedef struct {
  int32_t strip;        /* points per lane in the tile kernel's serial     */
                        /* strip hoods: 4, 8, 16 or 32 (0 = default 16)   */
  int32_t fan_in;       /* hoods merged per workgroup in a merge pass:     */
                        /* 2, 4, ..., 256 (0 = default: 256, or for a  */
                        /* plan of at least 8 tiles per compute unit 128  */
                        /* or 64 if needed for the first merge pass to    */
                        /* have an item per compute unit)                 */
  uint32_t flags;       /* UH_FLAG_* bits                                  */
} upper_hull_config;

#define UH_FLAG_FORCE_FALLBACK 1u /* every orientation takes the exact FP64 */
                                  /* path (ablation / soundness tests)      */
#define UH_FLAG_NO_VALIDATE 2u    /* skip the data-contract checks          */
#define UH_FLAG_GRAPH 4u          /* replay the run as a captured hipGraph  */
#define UH_FLAG_BOTH_HOODS 8u     /* also the lower hood of every set, from */
                                  /* the same single read of the points     */
                                  /* (output layout at upper_hull_plan_run) */
#define UH_FLAG_UNSORTED 16u      /* points of a set in any order: the plan */
                                  /* sorts every set by x on the device     */
                                  /* first (stable: equal x keep input      */
                                  /* order, so tie rules refer to input     */
                                  /* indices); corners are reported as      */
                                  /* input indices, left to right.  At most */
                                  /* 2^32 - 1 points; adds about 36 bytes   */
                                  /* per point of workspace.                */

/* ------------------------------------------------------------ single set */
/*
 * Upper hood of points[0..n).
 *   points    device, n float32 pairs (x, y), contract above.
 *   n         number of points, 0 <= n <= INT32_MAX.
 *   out_idx   device int32[n] (room for n: a strictly concave input makes
 *             every point a corner); the first *out_count entries are set.
 *   out_count device int32[1]: the corner count, or a negative data-error
 *             status.
 *   stream    HIP stream the work is enqueued on.
 * The library keeps a plan (schedule + workspace of about 12 bytes per
 * point) per distinct n, built on first use; building one is not allowed
 * while `stream` is capturing (UH_ERR_CAPTURE): call once before capture.
 * This is the paper's whole program (its stage loop and match_and_merge
 * launches) as one device-resident call.  Calls for the same n share that
 * plan's workspace, so calls on different streams must not overlap.
 */
int upper_hull(const float *points, int64_t n, int32_t *out_idx,
               int32_t *out_count, hipStream_t stream);

/*
 * Convex hull of points[0..n), the 2-D hull the paper's title and abstract
 * name: its corner indices counter-clockwise, starting at the lowest point of
 * least x (identical points resolve to the lowest index).  The lower hood is
 * the upper hood of the points mirrored in the x axis; both hoods come from
 * one read of the points (UH_FLAG_BOTH_HOODS), then the lower hood left to
 * right and the upper hood right to left, without the end corners the two
 * share, are joined into out_idx.
 *   points, n, stream   as for upper_hull.
 *   out_idx    device int32[n]: every index appears at most once.
 *   out_count  device int32[1]: the corner count, or a negative data-error
 *              status (the same checks as upper_hull).
 * Keeps its own cached plan per n (workspace about 24 bytes per point plus
 * 8 bytes per point of hood buffers); the same rules as upper_hull apply
 * (no plan building during capture, no overlapping calls for one n).
 */
int convex_hull(const float *points, int64_t n, int32_t *out_idx,
                int32_t *out_count, hipStream_t stream);

/* ------------------------------------------------------------ batched */
typedef struct upper_hull_plan upper_hull_plan;

/*
 * Build a plan for many independent point sets packed back to back: set s
 * is points[set_offsets[s] .. set_offsets[s+1]).
 *   set_offsets  HOST int64[num_sets + 1], non-decreasing, set_offsets[0]
 *                = 0; copied, the caller may free it afterwards.
 *   num_sets     >= 1.
 *   config       NULL for defaults.
 *   out_plan     receives the plan (owned by the caller; destroy it with
 *                upper_hull_plan_destroy).
 * Allocates the schedule tables and the workspace (about 12 bytes per point,
 * twice that with UH_FLAG_BOTH_HOODS,
 * plus a few bytes per tile) on the current device.
 */
int upper_hull_plan_create(const int64_t *set_offsets, int32_t num_sets,
                           const upper_hull_config *config,
                           upper_hull_plan **out_plan);

/*
 * Run a plan: hoods of all sets in one device-resident pass sequence.
 *   points      device, set_offsets[num_sets] float32 pairs.
 *   out_idx     device int32[set_offsets[num_sets]]; set s writes its
 *               corner indices (relative to set_offsets[s]) at
 *               out_idx + set_offsets[s].
 *   out_counts  device int32[num_sets]: corner count or data-error status.
 *   stats       device upper_hull_stats[num_sets] or NULL.
 *   stream      HIP stream.
 * With UH_FLAG_GRAPH the launch sequence is captured once per distinct
 * (points, out_idx, out_counts, stats) tuple and replayed as a hipGraph.
 * With UH_FLAG_BOTH_HOODS every array holds two halves: out_idx has
 * 2 * set_offsets[num_sets] entries, out_counts and stats 2 * num_sets; the
 * upper hoods fill the first half as above, and the lower hood of set s
 * (corners left to right, indices relative to set_offsets[s]) sits at
 * out_idx + set_offsets[num_sets] + set_offsets[s], its count at
 * out_counts[num_sets + s].  A data error is reported in both halves.
 */
int upper_hull_plan_run(upper_hull_plan *plan, const float *points,
                        int32_t *out_idx, int32_t *out_counts,
                        upper_hull_stats *stats, hipStream_t stream);

/*
 * Batched call without a plan object: upper hoods of all sets
 * points[set_offsets[s] .. set_offsets[s+1]) in one device-resident run,
 * with the default configuration.  Arguments and output layout as for
 * upper_hull_plan_create (set_offsets on the HOST) and upper_hull_plan_run.
 * The library keeps a plan per distinct set layout (a few, least recently
 * created dropped first), built on first use: not while `stream` is
 * capturing (UH_ERR_CAPTURE).  Calls with the same layout share that plan's
 * workspace, so calls on different streams must not overlap.
 */
int upper_hull_batched(const float *points, const int64_t *set_offsets, int32_t num_sets,
                       int32_t *out_idx, int32_t *out_counts, upper_hull_stats *stats,
                       hipStream_t stream);

/* Free a plan and its device memory (synchronises its device first). */
void upper_hull_plan_destroy(upper_hull_plan *plan);

/*
 * For a plan built with UH_FLAG_UNSORTED: the plan's own device buffers that
 * hold, after a run (once its stream has reached that point), every set's
 * points sorted by x (*sorted_points, float32 pairs, set s at
 * set_offsets[s]) and their set-relative input indices (*perm).  Owned by the
 * plan; overwritten by its next run.  UH_ERR_ARG for other plans.
 */
int upper_hull_plan_sorted(const upper_hull_plan *plan, const float **sorted_points,
                           const int32_t **perm);

/* The configuration a plan was built with, defaults resolved (strip,
 * fan_in, flags) into *config. */
int upper_hull_plan_config(const upper_hull_plan *plan, upper_hull_config *config);

/* Number of kernel launches one run of the plan enqueues (for profiling). */
int upper_hull_plan_launches(const upper_hull_plan *plan);

/*
 * Profiling hook: later runs of the plan record `before` on the run's
 * stream just before the tile kernel (the pass that reads every point) and
 * `after` just after it, so the caller can time that kernel alone with
 * hipEventElapsedTime.  Events are caller-created (hipEventCreate) and
 * caller-owned; pass NULL, NULL to stop.  Not available with UH_FLAG_GRAPH
 * (UH_ERR_ARG).
 */
int upper_hull_plan_set_probe(upper_hull_plan *plan, hipEvent_t before,
                              hipEvent_t after);

/*
 * Autotuner: chooses the tile size (T = 64 * strip points) and the number of
 * merge rounds fused per workgroup (log2 fan_in) for a set layout by timing
 * them on the caller's data.  Every (strip, fan_in) pair with strip in
 * {8, 16, 32} and fan_in in {16, 32, 64, 128, 256} runs `reps` times (after one
 * untimed run) on `stream` under `flags` (UH_FLAG_GRAPH is ignored); the
 * fastest mean time wins, ties to the earlier pair.  Synchronous: returns
 * when the timing is done.
 *   points, set_offsets, num_sets   as for a plan (points on the device,
 *                                    set_offsets on the host).
 *   flags     UH_FLAG_* bits to tune under; copied into *best.
 *   reps      1 .. 1000 timed runs per pair.
 *   best      receives the chosen config.
 *   best_ms   NULL, or receives its mean run time in milliseconds.
 * A data error in the sample (a negative count) does not stop the timing.
 * Builds a plan per pair and scratch output buffers while it runs and frees
 * them before returning: not for use while `stream` is capturing.
 */
int upper_hull_autotune(const float *points, const int64_t *set_offsets,
                        int32_t num_sets, uint32_t flags, int32_t reps,
                        upper_hull_config *best, float *best_ms,
                        hipStream_t stream);

/*
 * Measurement aid: the mean time (*ms) of a plain coalesced streaming read
 * of points[0 .. n) (whole 16-byte pairs; device, 16-byte aligned, n >= 2),
 * over `reps` launches (1 .. 1000) after one untimed launch on `stream`.
 * The tile kernel reads the same bytes, so 8 n / ms is the bandwidth a
 * simple read reaches on this device for this buffer.  Synchronous;
 * allocates 4 bytes of scratch while it runs.
 */
int upper_hull_read_reference(const float *points, int64_t n, int32_t reps, float *ms,
                              hipStream_t stream);

/* ------------------------------------------------------- building blocks */
/*
 * The bridge of two hoods (match-and-merge, steps mam1-mam5 of the paper,
 * with the tangent classifiers g and f): P and Q are the corner lists of
 * two strict upper hoods (device float32 pairs, strictly increasing x,
 * strictly concave), every P corner strictly left of every Q corner,
 * hp, hq >= 1.  Writes out_ab[0] = a, the leftmost P-corner on the common
 * tangent, and out_ab[1] = b, the rightmost Q-corner on it (device
 * int32[2]); the merged hood is P[0..a] followed by Q[b..hq).  `lanes`
 * (1, 2, 4, ..., 64) is the number of wave lanes the search uses, as in the
 * paper's d1 x d2 thread block.
 */
int upper_hull_bridge(const float *P, int32_t hp, const float *Q, int32_t hq,
                      int32_t lanes, int32_t *out_ab, hipStream_t stream);

/*
 * Orientation predicate (the paper's left_of, as a three-way sign): for
 * each i < m, out_sign[i] = sign of det(b_i - a_i, c_i - a_i), i.e. +1 when
 * c_i is left of (above, when a_i.x < b_i.x) the directed line a_i -> b_i.
 * a, b, c: device float32 pairs[m] on the data contract's grid and ranges;
 * out_sign: device int8[m]; out_fallback: device uint8[m] or NULL, set to 1
 * where the FP32 filter could not decide and the exact path was taken.
 * force_fallback != 0 sends every evaluation down the exact path.
 */
int upper_hull_orient(const float *a, const float *b, const float *c,
                      int64_t m, int8_t *out_sign, uint8_t *out_fallback,
                      int32_t force_fallback, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* WAGENER_HULL_H */
