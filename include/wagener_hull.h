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
#define UH_ERR_CAPTURE (-4)   /* device memory would have to be allocated  */
                              /* while the stream is being captured into a */
                              /* graph                                      */
#define UH_ERR_WORKSPACE (-5) /* the workspace set with                    */
                              /* upper_hull_set_workspace is too small for */
                              /* this call                                  */
#define UH_ERR_TOO_LARGE (-6) /* more points than upper_hull_noalloc's    */
                              /* fixed scratch serves (UH_NOALLOC_MAX_N)   */
#define UH_ERR_UNSORTED (-10) /* data: x decreases somewhere               */
#define UH_ERR_RANGE (-11)    /* data: x outside [0,1], y outside [-1,1],  */
                              /*       or a NaN / infinity                 */
#define UH_ERR_GRID (-12)     /* data: a coordinate is not on the 2^-30    */
                              /*       grid                                */

/* Human-readable text of a status code (static storage, never NULL). */
const char *upper_hull_status_string(int status);

/* Per-set counters written by the batched entry points (device memory). */
typedef struct {
  uint64_t orient_evals; /* orientation tests evaluated                    */
  uint64_t fallbacks;    /* of which the FP32 filter could not decide and  */
                         /* the exact FP64 evaluation was used             */
  uint64_t sign_errors;  /* with UH_FLAG_CHECK_SIGNS: tests whose sign     */
                         /* differed from a 128-bit integer evaluation     */
                         /* (0 on data that meets the contract)            */
  int32_t rounds;        /* rounds of pairwise merges over the set's       */
                         /* serial strip hoods of `strip` points:          */
                         /* ceil(log2(ceil(n / strip))), 0 for n <= strip; */
                         /* the strips stand for the paper's first         */
                         /* log2(strip) - 1 stages, which start at blocks  */
                         /* of two points                                  */
  int32_t status;        /* 0, or the set's negative data-error status     */
                         /* (the same value as its count)                  */
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
#define UH_FLAG_NO_ELIMINATION 32u /* no elimination of points before the   */
                                  /* merges: every point goes through the   */
                                  /* serial strip hoods and every round of  */
                                  /* Wagener merges (same result; for       */
                                  /* measuring the method itself and for    */
                                  /* upper_hull_plan_trace)                 */
#define UH_FLAG_CHECK_SIGNS 64u   /* soundness check: every orientation    */
                                  /* test is also evaluated in 128-bit      */
                                  /* integers; disagreements are counted in */
                                  /* upper_hull_stats.sign_errors (slow)    */

/* -------------------------------------------------------------- workspace */
/*
 * Device memory for the single-set calls (upper_hull and convex_hull).
 * Without a workspace set, the library keeps one per (device, stream),
 * allocated on first use and enlarged when a call needs more (allocation is
 * refused while the stream is capturing: UH_ERR_CAPTURE).  With a workspace
 * set, those calls allocate nothing, never synchronise the device and can be
 * captured into a graph for any size that fits.
 *
 * upper_hull_workspace_bytes: bytes that serve every call with at most
 * max_total_n points over at most max_sets sets (max_total_n >= 0,
 * max_sets >= 1): upper_hull of n points is one set of n points; convex_hull
 * of n points is two sets of n points (its upper and lower hood), so it needs
 * max_total_n >= 2 n and max_sets >= 2.  About 12 bytes per point plus small
 * tables.  Returns 0 for invalid arguments.
 *
 * upper_hull_set_workspace: from now on the single-set calls on the current
 * device use device_ptr[0 .. bytes) (256-byte aligned, caller-owned, not
 * freed by the library); a call it cannot serve returns UH_ERR_WORKSPACE and
 * enqueues nothing.  device_ptr = NULL, bytes = 0 goes back to library
 * memory.  Calls that use one workspace must not overlap in time (calls on
 * one stream never do); its contents between calls are the library's.
 * Synchronous; not while a stream of the device is capturing.
 */
size_t upper_hull_workspace_bytes(int64_t max_total_n, int32_t max_sets);
int upper_hull_set_workspace(void *device_ptr, size_t bytes);

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
 * The schedule follows from n (no table, nothing uploaded); the working
 * memory comes from the workspace (see upper_hull_set_workspace).  This is
 * the paper's whole program (its stage loop and match_and_merge launches) as
 * one device-resident call of two or three kernel launches.
 */
int upper_hull(const float *points, int64_t n, int32_t *out_idx,
               int32_t *out_count, hipStream_t stream);

/*
 * Upper hood of points[0..n) without any allocation, for callers that cannot
 * allocate device memory: code being captured into a graph, tight serving
 * loops, harnesses that forbid hipMalloc.  Arguments, result and errors as
 * for upper_hull; in addition n > UH_NOALLOC_MAX_N returns UH_ERR_TOO_LARGE
 * and enqueues nothing.
 * The working memory is a fixed device array inside the library (about
 * 12 bytes per point of UH_NOALLOC_MAX_N, 25 MB), one per device, held from
 * the library's first use on that device until the process ends; the call
 * never allocates, frees or synchronises.  Its device address is looked up
 * once per device, on the first call there (make that call outside a graph
 * capture).  Every call on a device shares that device's array, and each
 * call's last contents stay in it: calls that overlap in time on one device
 * (different streams, or different host threads without ordering) race and
 * give undefined results; calls on one stream never overlap.
 */
#define UH_NOALLOC_MAX_N (1 << 21)
int upper_hull_noalloc(const float *points, int64_t n, int32_t *out_idx,
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
 * Uses the workspace as upper_hull does, with two sets of n points (about
 * 28 bytes per point), plus one launch that joins the two hoods.
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
 * A plan owns its run's working memory, including per-set words that every
 * run leaves at zero for the next: runs of one plan must not overlap (keep
 * them on one stream, or order them with events).
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

/*
 * The blocks of one level of a plan's merge tree (level 0: the tiles of
 * 64 * strip points; level k >= 1: the blocks formed by merge pass k, each
 * the union of up to fan_in blocks of level k - 1 of one set; the last level
 * holds one block per set that needed that many passes).  Returns the number
 * of blocks (or UH_ERR_ARG for a level outside 0 .. number of passes); with
 * ranges != NULL (HOST int64[2 * blocks]) also block b's first point and
 * point count, in the plan's point numbering (with UH_FLAG_BOTH_HOODS the
 * lower hood of input point i is point set_offsets[num_sets] + i).
 */
int32_t upper_hull_plan_blocks(const upper_hull_plan *plan, int32_t level, int64_t *ranges);

/*
 * Debug trace of the merge tree, the paper's per-stage dump of every block's
 * hood: runs the plan's tile pass and its first `level` merge passes on
 * `points` (the whole run for the last level), then writes for every block b
 * of that level its corners' set-relative indices, left to right, at
 * out_idx + (block b's first point) and its count to out_counts[b].  With
 * UH_FLAG_NO_ELIMINATION every block then holds exactly the upper hood of its
 * points; otherwise blocks hold what survived the elimination, and a count
 * with bit 31 set marks a tile's sorted surviving points rather than a hood.
 *   out_idx     device int32[plan points] (both hoods: twice the points).
 *   out_counts  device int32[upper_hull_plan_blocks(plan, level, NULL)].
 * Not for UH_FLAG_UNSORTED plans.  Allocates a small buffer on first use.
 * Leaves the plan ready for normal runs.
 */
int upper_hull_plan_trace(upper_hull_plan *plan, const float *points, int32_t level,
                          int32_t *out_idx, int32_t *out_counts, hipStream_t stream);

/* The configuration a plan was built with, defaults resolved (strip,
 * fan_in, flags) into *config. */
int upper_hull_plan_config(const upper_hull_plan *plan, upper_hull_config *config);

/* Number of kernel launches one run of the plan enqueues (for profiling);
 * with_stats != 0: a run given a stats array (which adds the clearing
 * launch when no set is empty). */
int upper_hull_plan_launches(const upper_hull_plan *plan, int32_t with_stats);

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
