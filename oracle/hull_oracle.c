/*
 * Hood and hull oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU computation of what the GPU path
 * computes: the upper hood (upper convex hull, closed by downward vertical
 * rays) of a set of points given in left-to-right order, returned as the
 * input indices of its corners, left to right; the lower hood (its mirror
 * image under y -> -y); and the whole convex hull assembled from the two.  Only the tests, the smoke
 * check and the benchmark's CPU baseline may load this library; the product
 * path never calls it.  It shares no code, header or constant generator with
 * the GPU library.
 *
 * Paper: C. O Dunlaing, "CUDA implementation of Wagener's 2D convex hull PRAM
 * algorithm".  What is followed here:
 *   - problem statement (section "Wagener's algorithm, CUDA version"): the
 *     input is n points in left-to-right order with x in [0, 1]; the output
 *     is the upper hood of the set;
 *   - orientation convention (the left_of predicate described just before
 *     the g and f classifiers): r is left of the directed segment pq iff
 *     det(q - p, r - p) > 0; with p.x < q.x "left" means "above";
 *   - vertical closure: the classifiers g and f treat a missing neighbour
 *     as a point directly below the end corner, i.e. the hood is closed by
 *     downward vertical rays, so at any x only the highest point can be a
 *     corner.
 *
 * Readings where the paper is silent (it assumes no three points collinear,
 * n a power of two, and no floating-point error):
 *   - strict hood: a point in the relative interior of a hood edge is not a
 *     corner (pop while orient >= 0);
 *   - equal x: only the highest point of a run of equal x can be a corner;
 *     identical points resolve to the lowest index;
 *   - exactness: coordinates are read as exact integers on the 2^-30 grid
 *     (every float32 in [2^-7, 1] is on it), orientation is evaluated in
 *     128-bit integers, so every sign is exact;
 *   - any n >= 0 is accepted.
 *
 * Algorithm (Andrew's monotone chain, upper half), steps in order:
 *   1. convert each coordinate to an exact integer, validating the contract;
 *   2. keep one representative per run of equal x (max y, lowest index);
 *   3. scan representatives left to right, popping the stack top while the
 *      new point is on or above the line through the top two, then push.
 *
 * Lower hood and convex hull (the paper's title and abstract promise the 2-D
 * convex hull; the method it details builds the upper hood only):
 *   - the lower hood of a set is the reflection, under y -> -y, of the upper
 *     hood of the reflected set, corner indices unchanged: at an x only the
 *     lowest point can be a corner (ties to the lowest index), and a point on
 *     or above the line through its neighbours is dropped;
 *   - the convex hull, counter-clockwise from the lowest point of least x, is
 *     the lower hood left to right followed by the upper hood right to left,
 *     each hood's end corner omitted where the two hoods share it.
 *
 * The chain's correctness is not taken on trust: the tests pin it against an
 * O(n^3) brute-force evaluation of the hood's definition, against Qhull on
 * points in general position, and against closed forms and invariants.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef __int128 i128;

/* status codes (values mirror the library's documented contract) */
#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_UNSORTED (-10)
#define OR_ERR_RANGE (-11)
#define OR_ERR_GRID (-12)

#define GRID_SCALE 1073741824.0 /* 2^30 */

/* Step 1: exact integer coordinate on the 2^-30 grid.  Returns 0 or an
 * error code.  x must lie in [0, 1], y in [-1, 1]; NaN fails the range test. */
static int grid_int(float v, double lo, double hi, int64_t *out) {
  double d = (double)v;
  if (!(d >= lo && d <= hi)) return OR_ERR_RANGE;
  double s = d * GRID_SCALE; /* exact: power-of-two scaling of a float */
  double t = floor(s);
  if (t != s) return OR_ERR_GRID;
  *out = (int64_t)t;
  return OR_OK;
}

/* det(b - a, c - a): > 0 iff c is left of (above) the directed line a->b. */
static i128 orient(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx,
                   int64_t cy) {
  return (i128)(bx - ax) * (i128)(cy - ay) - (i128)(by - ay) * (i128)(cx - ax);
}

/* Validate and convert all points; returns 0 or an error code. */
static int convert(const float *xy, int64_t n, int64_t *X, int64_t *Y) {
  for (int64_t i = 0; i < n; ++i) {
    int rc = grid_int(xy[2 * i], 0.0, 1.0, &X[i]);
    if (rc) return rc;
    rc = grid_int(xy[2 * i + 1], -1.0, 1.0, &Y[i]);
    if (rc) return rc;
    if (i > 0 && X[i] < X[i - 1]) return OR_ERR_UNSORTED;
  }
  return OR_OK;
}

/* Steps 2-3 on already converted coordinates.  idx_base is added to the
 * written indices (0 for a single set).  Returns the corner count. */
static int64_t chain(const int64_t *X, const int64_t *Y, int64_t n,
                     int32_t *out_idx) {
  int64_t h = 0; /* out_idx doubles as the stack */
  int64_t i = 0;
  while (i < n) {
    /* step 2: representative of the run of equal x starting at i */
    int64_t rep = i, j = i + 1;
    while (j < n && X[j] == X[i]) {
      if (Y[j] > Y[rep]) rep = j; /* strict: ties keep the lowest index */
      ++j;
    }
    i = j;
    /* step 3: pop while the new point is on or above line (h-2, h-1) */
    while (h >= 2) {
      int64_t a = out_idx[h - 2], b = out_idx[h - 1];
      if (orient(X[a], Y[a], X[b], Y[b], X[rep], Y[rep]) >= 0)
        --h;
      else
        break;
    }
    out_idx[h++] = (int32_t)rep;
  }
  return h;
}

/* The upper hood (lower = 0) or the lower hood (lower = 1) of xy[0..n):
 * the lower hood is the upper hood of the points reflected in the x axis. */
static int hood(const float *xy, int64_t n, int32_t *out_idx, int64_t *out_count,
                int lower) {
  if (n < 0 || n > INT32_MAX || (n > 0 && (!xy || !out_idx)) || !out_count)
    return OR_ERR_ARG;
  *out_count = 0;
  if (n == 0) return OR_OK;
  int64_t *X = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t *Y = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  if (!X || !Y) {
    free(X);
    free(Y);
    return OR_ERR_ARG;
  }
  int rc = convert(xy, n, X, Y);
  if (rc == OR_OK && lower)
    for (int64_t i = 0; i < n; ++i) Y[i] = -Y[i];
  if (rc == OR_OK) *out_count = chain(X, Y, n, out_idx);
  free(X);
  free(Y);
  return rc;
}

/* Upper hood of xy[0..n) (x, y interleaved float32).  out_idx needs room for
 * n entries.  Returns 0 and sets *out_count, or a negative error code. */
int oracle_upper_hull(const float *xy, int64_t n, int32_t *out_idx,
                      int64_t *out_count) {
  return hood(xy, n, out_idx, out_count, 0);
}

/* Lower hood of xy[0..n), corner indices left to right; as above. */
int oracle_lower_hull(const float *xy, int64_t n, int32_t *out_idx,
                      int64_t *out_count) {
  return hood(xy, n, out_idx, out_count, 1);
}

/* Convex hull of xy[0..n): corner indices counter-clockwise, starting at the
 * lowest point of least x (lowest index among identical points).  out_idx
 * needs room for n entries (every index appears at most once). */
int oracle_convex_hull(const float *xy, int64_t n, int32_t *out_idx,
                       int64_t *out_count) {
  if (n < 0 || n > INT32_MAX || (n > 0 && (!xy || !out_idx)) || !out_count)
    return OR_ERR_ARG;
  *out_count = 0;
  if (n == 0) return OR_OK;
  int32_t *up = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!up) return OR_ERR_ARG;
  int64_t hl = 0, hu = 0;
  int rc = hood(xy, n, out_idx, &hl, 1); /* lower hood, left to right */
  if (rc == OR_OK) rc = hood(xy, n, up, &hu, 0);
  if (rc == OR_OK) {
    int64_t h = hl;
    for (int64_t k = hu - 1; k >= 0; --k) { /* upper hood, right to left */
      if (k == hu - 1 && up[k] == out_idx[hl - 1]) continue; /* shared right end */
      if (k == 0 && up[k] == out_idx[0]) continue;           /* shared left end */
      out_idx[h++] = up[k];
    }
    *out_count = h;
  }
  free(up);
  return rc;
}

/* Many independent sets: set s is xy[offsets[s] .. offsets[s+1]); its corner
 * indices (relative to offsets[s]) are written at out_idx + offsets[s] and
 * its count to out_counts[s].  Returns 0 or the first error code; a set
 * that fails gets its error code as its count. */
static int batched(const float *xy, const int64_t *offsets, int64_t num_sets,
                   int32_t *out_idx, int64_t *out_counts, int lower) {
  if (num_sets < 0 || !offsets || (num_sets > 0 && !out_counts))
    return OR_ERR_ARG;
  int first_err = OR_OK;
  for (int64_t s = 0; s < num_sets; ++s) {
    int64_t lo = offsets[s], hi = offsets[s + 1];
    int64_t cnt = 0;
    int rc = hood(xy + 2 * lo, hi - lo, out_idx + lo, &cnt, lower);
    out_counts[s] = rc ? rc : cnt;
    if (rc && !first_err) first_err = rc;
  }
  return first_err;
}

int oracle_upper_hull_batched(const float *xy, const int64_t *offsets,
                              int64_t num_sets, int32_t *out_idx,
                              int64_t *out_counts) {
  return batched(xy, offsets, num_sets, out_idx, out_counts, 0);
}

int oracle_lower_hull_batched(const float *xy, const int64_t *offsets,
                              int64_t num_sets, int32_t *out_idx,
                              int64_t *out_counts) {
  return batched(xy, offsets, num_sets, out_idx, out_counts, 1);
}

/* Exact sign of det(b - a, c - a) for m triples of float points (each array
 * holds x, y interleaved).  Writes -1, 0 or +1.  Returns 0 or an error code
 * (off-grid or out-of-range coordinate). */
int oracle_orient_signs(const float *a, const float *b, const float *c,
                        int64_t m, int8_t *out_sign) {
  for (int64_t i = 0; i < m; ++i) {
    int64_t v[6];
    const float *src[3] = {a + 2 * i, b + 2 * i, c + 2 * i};
    for (int k = 0; k < 3; ++k) {
      int rc = grid_int(src[k][0], 0.0, 1.0, &v[2 * k]);
      if (rc) return rc;
      rc = grid_int(src[k][1], -1.0, 1.0, &v[2 * k + 1]);
      if (rc) return rc;
    }
    i128 d = orient(v[0], v[1], v[2], v[3], v[4], v[5]);
    out_sign[i] = (int8_t)((d > 0) - (d < 0));
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------
 * All-cores variants, for the CPU baseline's timing only.
 *
 * The same chain, split over threads, relying on one fact of the hood's
 * definition: a point that is no corner of the hood of a subset holding it
 * (it lies on or below a segment between two points of the subset, or below
 * a point of the subset at its x) is no corner of the hood of the whole set
 * either.  So the hood of a set cut into x-ordered chunks is the hood of the
 * union of the chunks' hoods.  Chunk cuts are moved forward to the start of
 * a run of equal x, so every run lies in one chunk and its representative is
 * chosen exactly as in the single chain.  Each thread validates, converts
 * and chains one chunk; one final chain over the concatenated chunk hoods
 * (still in x order) gives the result.  Data errors are reported for the
 * lowest failing index, with the checks of one point taken in the order of
 * the single-threaded `convert`.
 * ---------------------------------------------------------------------- */
typedef struct {
  const float *xy;
  int64_t lo, hi;     /* the chunk's points [lo, hi) */
  int64_t *X, *Y;     /* whole-set buffers; this job fills [lo, hi) */
  int32_t *hood_idx;  /* the chunk's hood, chunk-relative, at hood_idx + lo */
  int64_t count;
  int64_t err_pos;    /* lowest failing index in the chunk, -1 if none */
  int err;
  int lower;
} chunk_job;

static void *chunk_main(void *arg) {
  chunk_job *j = (chunk_job *)arg;
  j->err = OR_OK;
  j->err_pos = -1;
  j->count = 0;
  for (int64_t i = j->lo; i < j->hi; ++i) {
    int rc = grid_int(j->xy[2 * i], 0.0, 1.0, &j->X[i]);
    if (!rc) rc = grid_int(j->xy[2 * i + 1], -1.0, 1.0, &j->Y[i]);
    if (!rc && i > 0) {
      int64_t prev = 0;
      if (i > j->lo)
        prev = j->X[i - 1];
      else if (grid_int(j->xy[2 * i - 2], 0.0, 1.0, &prev))
        prev = INT64_MIN; /* the previous chunk reports that point's error */
      if (j->X[i] < prev) rc = OR_ERR_UNSORTED;
    }
    if (rc) {
      j->err = rc;
      j->err_pos = i;
      return NULL;
    }
  }
  if (j->lower)
    for (int64_t i = j->lo; i < j->hi; ++i) j->Y[i] = -j->Y[i];
  j->count = chain(j->X + j->lo, j->Y + j->lo, j->hi - j->lo, j->hood_idx + j->lo);
  return NULL;
}

static int hood_mt(const float *xy, int64_t n, int32_t nthreads, int32_t *out_idx,
                   int64_t *out_count, int lower) {
  if (n < 0 || n > INT32_MAX || (n > 0 && (!xy || !out_idx)) || !out_count || nthreads < 1 ||
      nthreads > 1024)
    return OR_ERR_ARG;
  *out_count = 0;
  if (n == 0) return OR_OK;
  int64_t T = nthreads;
  if (T > n) T = n;
  int64_t *X = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t *Y = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int32_t *hidx = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  chunk_job *jobs = (chunk_job *)calloc((size_t)T, sizeof(chunk_job));
  pthread_t *tid = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
  int rc = OR_OK;
  if (!X || !Y || !hidx || !jobs || !tid) rc = OR_ERR_ARG;
  if (rc == OR_OK) {
    /* cuts: nominal k n / T, moved forward past a run of equal x */
    int64_t lo = 0;
    for (int64_t k = 0; k < T; ++k) {
      int64_t hi = k + 1 == T ? n : (k + 1) * n / T;
      if (hi < lo) hi = lo;
      while (hi < n && hi > 0 && xy[2 * hi] == xy[2 * hi - 2]) ++hi;
      jobs[k] = (chunk_job){xy, lo, hi, X, Y, hidx, 0, -1, OR_OK, lower};
      lo = hi;
    }
    int64_t started = 0;
    for (int64_t k = 1; k < T; ++k) {
      if (pthread_create(&tid[k], NULL, chunk_main, &jobs[k]) != 0) break;
      started = k;
    }
    chunk_main(&jobs[0]);
    for (int64_t k = started + 1; k < T; ++k) chunk_main(&jobs[k]); /* not started */
    for (int64_t k = 1; k <= started; ++k) pthread_join(tid[k], NULL);
    for (int64_t k = 0; k < T; ++k)
      if (jobs[k].err) { /* the lowest failing index is in the earliest failing chunk */
        rc = jobs[k].err;
        break;
      }
  }
  if (rc == OR_OK) {
    /* the final chain over the chunk hoods, in x order */
    int64_t m = 0;
    for (int64_t k = 0; k < T; ++k)
      for (int64_t e = 0; e < jobs[k].count; ++e) {
        const int64_t g = jobs[k].lo + hidx[jobs[k].lo + e];
        X[m] = X[g];
        Y[m] = Y[g];
        out_idx[m] = (int32_t)g; /* candidate m's input index */
        ++m;
      }
    int32_t *pos = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!pos) {
      rc = OR_ERR_ARG;
    } else {
      const int64_t h = chain(X, Y, m, pos);
      for (int64_t e = 0; e < h; ++e) pos[e] = out_idx[pos[e]];
      memcpy(out_idx, pos, (size_t)h * sizeof(int32_t));
      *out_count = h;
      free(pos);
    }
  }
  free(X);
  free(Y);
  free(hidx);
  free(jobs);
  free(tid);
  return rc;
}

/* Upper hood (lower = 0) or lower hood (lower = 1) of xy[0..n) on nthreads
 * threads (1 .. 1024); the same result and status as oracle_upper_hull /
 * oracle_lower_hull. */
int oracle_hood_mt(const float *xy, int64_t n, int32_t nthreads, int32_t lower,
                   int32_t *out_idx, int64_t *out_count) {
  return hood_mt(xy, n, nthreads, out_idx, out_count, lower != 0);
}

typedef struct {
  const float *xy;
  const int64_t *offsets;
  int64_t num_sets;
  int32_t *out_idx;
  int64_t *out_counts;
  int lower;
  int64_t next; /* next set to take (atomic) */
} sets_job;

static void *sets_main(void *arg) {
  sets_job *j = (sets_job *)arg;
  for (;;) {
    const int64_t s = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
    if (s >= j->num_sets) return NULL;
    const int64_t lo = j->offsets[s], hi = j->offsets[s + 1];
    int64_t cnt = 0;
    const int rc = hood(j->xy + 2 * lo, hi - lo, j->out_idx + lo, &cnt, j->lower);
    j->out_counts[s] = rc ? rc : cnt;
  }
}

/* Many sets on nthreads threads, each set's chain on one thread (sets taken
 * in index order as threads become free); the same layout and per-set
 * statuses as oracle_upper_hull_batched / oracle_lower_hull_batched.
 * Returns 0 or the status of the lowest-numbered failing set. */
int oracle_hood_batched_mt(const float *xy, const int64_t *offsets, int64_t num_sets,
                           int32_t nthreads, int32_t lower, int32_t *out_idx,
                           int64_t *out_counts) {
  if (num_sets < 0 || !offsets || (num_sets > 0 && !out_counts) || nthreads < 1 ||
      nthreads > 1024)
    return OR_ERR_ARG;
  sets_job job = {xy, offsets, num_sets, out_idx, out_counts, lower != 0, 0};
  pthread_t tid[1024];
  int32_t started = 0;
  for (int32_t k = 1; k < nthreads; ++k) {
    if (pthread_create(&tid[k], NULL, sets_main, &job) != 0) break;
    started = k;
  }
  sets_main(&job);
  for (int32_t k = 1; k <= started; ++k) pthread_join(tid[k], NULL);
  for (int64_t s = 0; s < num_sets; ++s)
    if (out_counts[s] < 0) return (int)out_counts[s];
  return OR_OK;
}

/* Threads available to this process (the CPU baseline reports it). */
int32_t oracle_online_cpus(void) { return (int32_t)sysconf(_SC_NPROCESSORS_ONLN); }
