/*
 * kp.h -- C ABI of the MI355X (gfx950) filtered K-means library (libkp.so).
 *
 * The library runs the K-means iteration of KPynq (Wang et al., "KPynq: A
 * Work-Efficient Triangle-Inequality based K-means on FPGA"): a point-level
 * filter, then a group-level filter, then a distance calculator for the
 * (point, centroid group) pairs that survive, then the centroid update
 * (Section 1 names the filters and the distance calculator; the Abstract
 * states that the result is that of standard K-means).  Every stage is a HIP
 * kernel for gfx950; the host code here only plans memory, groups the
 * centroids once at kp_init and launches work on a stream.
 *
 * Conventions shared by every call:
 *  - Pointers named *_dev are device pointers (HBM of the ctx's GPU).  Host
 *    pointers are named *_host.  No call keeps a host pointer.
 *  - The caller owns every buffer: the points, the workspace and all
 *    outputs.  The library never allocates device memory; all of its state
 *    lives in the caller's workspace (kp_workspace_bytes).  It allocates
 *    small host-side bookkeeping only in kp_init.
 *  - Matrices are row-major FP32 with no padding: point i of problem p is
 *    points_dev[i*d .. i*d+d-1].
 *  - Centroid indices at the boundary are the caller's original indices
 *    0..k-1; ties between equally near centroids go to the lowest index.
 *  - Every call returns a kp_status.  KP_ERR_INVALID (bad argument) leaves
 *    the ctx unchanged.  KP_ERR_HIP (a HIP runtime failure) poisons the ctx:
 *    every later call except kp_destroy returns KP_ERR_STATE.
 *    kp_last_error() gives a detail string for the calling thread.
 *  - A ctx is bound to one device and one stream and is not thread-safe.
 *    Work is ordered after everything already queued on that stream and
 *    everything later queued on it runs after it.
 */
#ifndef KP_H
#define KP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kp_ctx kp_ctx;   /* opaque */

typedef enum {
    KP_OK = 0,
    KP_ERR_INVALID = 1,      /* bad size, NULL, short or misaligned workspace */
    KP_ERR_NOMEM = 2,        /* host allocation failed */
    KP_ERR_HIP = 3,          /* HIP runtime error; the ctx is poisoned */
    KP_ERR_STATE = 4,        /* call on a poisoned ctx, or out of order */
    KP_ERR_UNSUPPORTED = 5   /* valid request outside what this build supports */
} kp_status;

typedef enum {
    /* Distances in FP32, direct form sum (x_i - c_i)^2 on the vector ALUs. */
    KP_PREC_FP32 = 0,
    /* Distances as ||x||^2 - 2 x.c + ||c||^2 with x and c rounded to BF16 on
     * MFMA (FP32 accumulation); every point whose decision is not certain
     * under the derived error bound is re-checked in FP32 direct form.
     * Centroid sums, means and drifts are FP64 in both modes. */
    KP_PREC_BF16_RECHECK = 1
} kp_precision;

/* One K-means problem. */
typedef struct {
    int64_t n;                     /* points, 1 <= k <= n < 2^31 */
    int32_t d;                     /* dimensions: kp_workspace_bytes accepts
                                      1 <= d <= 1024; kp_init supports
                                      d <= 128 in FP32 mode and d <= 256 in
                                      BF16 mode and returns
                                      KP_ERR_UNSUPPORTED above that */
    int32_t k;                     /* centroids, 1 <= k <= 65536 */
    int32_t g;                     /* centroid groups, 1 <= g <= k; BF16 mode
                                      supports g <= 1024 (KP_ERR_UNSUPPORTED
                                      from kp_init above that) */
    int32_t precision;             /* kp_precision */
    const float *points_dev;       /* n*d FP32; BORROWED: must stay valid and
                                      unchanged until kp_destroy */
    const float *init_centroids_dev; /* k*d FP32; copied during kp_init */
    uint64_t seed;                 /* seeds the grouping of the centroids */
} kp_problem;

/* Launch tuning.  Pass NULL for the built-in defaults.  A zero field means
 * "default" for that field. */
typedef struct {
    int32_t waves_per_block;       /* 1..4 waves of 64 lanes per workgroup */
    int32_t blocks_per_cu;         /* grid = 256 CUs * this (grid-stride loops) */
    int32_t use_graph;             /* 1 (default): replay each filtered
                                      iteration from a captured hipGraph;
                                      2: every iteration of a kp_iterate call
                                      (the dense first one included) in one
                                      graph, captured on the first call of
                                      that iteration count and replayed by
                                      later ones (requires timing = 0);
                                      -1: plain launches */
    int32_t timing;                /* 1: record HIP events on the ctx's stream
                                      around every stage of timing_stages
                                      (also inside graph replays) and around
                                      every replay (kp_stage_times); 0: none */
    int32_t chunk_depth;           /* BF16 mode: centroid chunks in flight per
                                      workgroup in the filtered distance pass,
                                      1 or 3 (default 1; the dense first pass
                                      always keeps 3) */
    int32_t bound_codes;           /* BF16 mode: per-(point, group) lower
                                      bounds stored as 1 = FP32 (default) or
                                      2 = FP16 codes rounded down (half the
                                      bound bytes, bounds up to 2^-10 looser;
                                      kp_workspace_bytes shrinks accordingly) */
    int32_t timing_stages;         /* with timing = 1: bit s brackets stage s
                                      with events, s = 0 "begin", 1
                                      "bound_filter", 2 "l1_sort", 3
                                      "assign_dense", 4 "group_filter", 5
                                      "assign", 6 "recheck", 7 "update", 8
                                      "centroids"; 0: every stage.  Whole
                                      replays are always timed */
    int32_t deterministic;         /* 1: bitwise reproducible runs.  The list
                                      of points failing the point-level filter
                                      is compacted in point order and sorted
                                      stably, and each update recomputes the
                                      FP64 centroid sums from all points in a
                                      fixed order (points sorted by centroid,
                                      then by index) with no floating-point
                                      atomics, so two runs of the same
                                      problems on the same device give the
                                      same labels, centroids and statistics
                                      bit for bit.  0 (default): incremental
                                      sums over the moved points with FP64
                                      atomic adds, whose order varies */
    int32_t local_filter;          /* FP32 problems: 1 = the per-centroid local
                                      filter inside each open group (a member
                                      is skipped when its group's bound, raised
                                      by how much less than the group's largest
                                      drift it moved, exceeds ub for every
                                      point of the 64-point tile that visits
                                      the group).  0 (default): every member of
                                      an open group is computed, which keeps
                                      the group bounds exact and, on the
                                      workloads measured, is faster overall */
    int32_t plain;                 /* 1: plain Lloyd, the comparator of the
                                      filtered method: every iteration
                                      computes every distance (the dense pass
                                      of the first iteration, with plain
                                      launches) and recomputes the centroid
                                      sums from all points; no filter skips
                                      anything.  0 (default): the filtered
                                      iterations of Section 1 */
} kp_tuning;

/* Per-iteration counters of one problem (kp_stats). */
typedef struct {
    int32_t iter;                  /* 1-based iteration number */
    int32_t dense;                 /* 1 if this iteration computed all distances */
    int64_t point_filter_fail;     /* points whose upper bound reached the point-level lower bound
                                      (and, with row_test, some group's bound): list L1 */
    int64_t pairs;                 /* (point, group) pairs that survived the group-level filter */
    int64_t distances;             /* point-centroid distances computed (padding excluded) */
    int64_t rechecks;              /* points re-decided in FP32 direct form */
    int64_t moved;                 /* points whose assignment changed */
    double max_drift;              /* largest centroid move of this iteration's update */
    int64_t tile_groups;           /* (64-point tile, open group) pairs visited by the distance kernel */
    int64_t closed;                /* points with every group bound closed, their own group's
                                      included: dropped from the point-filter failures by the
                                      row test when it ran, else found by the group filter */
    int32_t row_test;              /* 1 if the point-level filter tested whole bound rows in this
                                      iteration (on after an iteration with closed >= n / 8) */
    int32_t pad_;
} kp_iter_stats;

/* Accumulated GPU time of one stage (kp_stage_times). */
typedef struct {
    char name[24];                 /* "assign_dense", "bound_filter", "l1_sort",
                                      "group_filter" (BF16 mode), "assign", "recheck",
                                      "update", "centroids", "begin", "filtered_iter" */
    double ms;                     /* total milliseconds between the stage's events */
    int64_t launches;              /* number of timed launches */
} kp_stage_time;

/* Bytes of device workspace kp_init needs for these problems; 0 if the
 * description is invalid (kp_last_error says why).  The workspace holds the
 * per-point state of the filters (Section 1: the point-level filter's
 * per-point bounds, the group-level filter's per-(point, group) bounds) and
 * the centroid tables; its size grows with n * g. */
size_t kp_workspace_bytes(const kp_problem *problems_host, int32_t count, const kp_tuning *tuning_host);

/* Validate the problems, carve the workspace, group each problem's
 * centroids (host, once: the centroid groups the group-level filter of
 * Section 1 works on) and queue the per-point preparation on `stream`
 * (a hipStream_t; NULL = the default stream).  Synchronises the stream.
 * workspace_dev must be 256-byte aligned and hold kp_workspace_bytes().
 * On success *out receives a new ctx. */
kp_status kp_init(kp_ctx **out, const kp_problem *problems_host, int32_t count,
                  void *workspace_dev, size_t workspace_bytes, void *stream,
                  const kp_tuning *tuning_host);

/* Queue `iters` K-means iterations (assignment step + centroid update) of
 * every problem on the ctx stream; returns without waiting.  This is the
 * method of Section 1 and Fig. 1: a point-level filter, a group-level
 * filter, a distance calculator for the (point, group) pairs that are not
 * filtered out, then the centroid update; the Abstract states that the
 * result is that of standard K-means (Lloyd's algorithm), reached with fewer
 * distance computations.  The first iteration of a ctx computes every
 * distance (no bounds exist yet); later ones are filtered.  iters must be
 * >= 1 (KP_ERR_INVALID otherwise); a HIP launch failure returns KP_ERR_HIP
 * and poisons the ctx. */
kp_status kp_iterate(kp_ctx *ctx, int32_t iters);

/* Queue a copy of problem `problem`'s current assignment (n int32, original
 * centroid indices) to labels_dev: the output of the assignment step of
 * standard K-means (Abstract; Section 2 compares against it).
 * KP_ERR_STATE before the first iteration; KP_ERR_INVALID for a bad
 * problem index or NULL labels_dev. */
kp_status kp_assign(kp_ctx *ctx, int32_t problem, int32_t *labels_dev);

/* Queue a copy of problem `problem`'s current centroids (k*d, original order)
 * as FP32 (the values distances use) and/or FP64 (the exact means); either
 * pointer may be NULL.  These are the means of the update step of standard
 * K-means (Abstract); a centroid that received no point keeps its value.
 * KP_ERR_INVALID for a bad problem index. */
kp_status kp_centroids(kp_ctx *ctx, int32_t problem, float *c32_dev, double *c64_dev);

/* Synchronise the ctx stream and copy up to `cap` per-iteration records of
 * problem `problem` (oldest first) to stats_host; *n_host receives the count
 * written.  At most the last 1024 iterations are kept.  The records count
 * what each filter level of Section 1 left to the distance calculator.
 * KP_ERR_INVALID for a bad index, a negative cap or NULL outputs. */
kp_status kp_stats(kp_ctx *ctx, int32_t problem, kp_iter_stats *stats_host, int32_t cap, int32_t *n_host);

/* With kp_tuning.timing = 1: synchronise the ctx stream and return, per
 * stage, the GPU time measured by HIP events recorded on the ctx's internal
 * stream immediately before and after the stage's kernels, summed over all
 * iterations queued so far.  Stages replayed inside a hipGraph are timed as
 * one "filtered_iter" entry per replay.  Writes up to `cap` entries to
 * out_host and their count to *n_host.  KP_ERR_STATE when timing is off. */
kp_status kp_stage_times(kp_ctx *ctx, kp_stage_time *out_host, int32_t cap, int32_t *n_host);

/* Number of iterations completed on the ctx (host-side count of queued
 * iterations).  Returns -1 for NULL. */
int32_t kp_iterations(const kp_ctx *ctx);

/* Serving: bytes of device scratch kp_predict needs for nq query points
 * (the assignment step of Section 1 applied to new points)
 * (0 with kp_last_error set for a NULL ctx, a bad problem index or nq outside
 * 0..2^31-1). */
size_t kp_predict_scratch_bytes(const kp_ctx *ctx, int32_t problem, int64_t nq);

/* Serving: queue the assignment of nq new points (queries_dev: nq*d FP32,
 * row-major, 16-byte aligned; read until the queued work completes) to the
 * current centroids of problem `problem` -- the assignment step of the
 * iteration (Section 1) applied to points outside the training set, with its
 * decision rule: labels_dev[i] receives the original index of the nearest
 * centroid, ties to the lowest index.  BF16 problems decide on the BF16x3
 * estimate under its error bound.  With anchor tables (at most 16384 slots)
 * every query is first estimated relative to its nearest chunk medoid
 * (queries sorted by it), the uncertain ones again relative to their
 * provisional nearest centroid, and those still uncertain are recomputed in
 * FP32 direct form over every centroid; without, one plain BF16 pass comes
 * before the FP32 one.  FP32 problems use the FP32 direct form.
 * Before the first iteration the initial centroids are used.  Nothing of the
 * problem's state changes.  scratch_dev: caller-owned device memory of
 * kp_predict_scratch_bytes(), 256-byte aligned, overwritten.  Ordered on the
 * ctx's stream like kp_assign.  nq = 0 is a no-op; KP_ERR_INVALID for a bad
 * problem index, NULL or misaligned pointers or short scratch. */
kp_status kp_predict(kp_ctx *ctx, int32_t problem, const float *queries_dev, int64_t nq, int32_t *labels_dev,
                     void *scratch_dev, size_t scratch_bytes);

/* Serving for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): as
 * kp_predict, but the scratch is a fixed array the library holds on each
 * device it runs on (until the process ends), so the call allocates nothing.
 * nq may be at most KP_PREDICT_NOALLOC_MAX_QUERIES (KP_ERR_INVALID above it;
 * the array is about 64 MiB: 16 bytes per query and a slot histogram).
 * Every call on one device shares that device's array, whose counters and
 * histogram each call clears before use: calls that
 * overlap on one device (other streams or threads) race and must not be
 * issued.  Same labels as kp_predict; same argument errors. */
#define KP_PREDICT_NOALLOC_MAX_QUERIES 4194304
kp_status kp_predict_noalloc(kp_ctx *ctx, int32_t problem, const float *queries_dev, int64_t nq,
                             int32_t *labels_dev);

/* Synchronise and release the ctx's host resources, stream and graph.  The
 * workspace and points are the caller's to free afterwards.  NULL is a
 * no-op. */
kp_status kp_destroy(kp_ctx *ctx);

/* Autotuner of the launch shapes (the batched form picks its tiles and
 * workgroups per problem from it) -- the counterpart of the tunable
 * parameters, such as the degree of parallelism, of Section 1.  Runs `iters`
 * iterations (>= 2) of the problems from their initial centroids under each
 * candidate tuning --
 * bound storage {FP32, FP16} (BF16 problems) x centroid chunks in flight
 * {1, 3} x workgroups per CU {8, 16, 32} -- in the
 * caller's workspace (kp_workspace_bytes of the same problems with a NULL
 * tuning, the FP32-bound size), timing each
 * run with HIP events on `stream`, and writes the fastest to *best_host
 * (use_graph 1, timing 0).  Synchronises `stream`; leaves no ctx behind.
 * The workspace contents are undefined afterwards. */
kp_status kp_autotune(const kp_problem *problems_host, int32_t count, void *workspace_dev,
                      size_t workspace_bytes, void *stream, int32_t iters, kp_tuning *best_host);

/* Autotuner of the group counts.  The result of the method does not depend
 * on g (the filters of Section 1 only skip distances that cannot change an
 * assignment), so g is a speed parameter like the degree of parallelism of
 * Section 1.  For each class of problems with the same (d, k, precision), in
 * the order of first appearance, runs `iters` iterations (>= 2) of that
 * class's problems from their initial centroids under each candidate:
 * every problem's own g, ceil(k / 16) (the fewest groups that each fit one
 * 16-slot tile of the BF16 distance kernels) and ceil(k / 10), each clipped
 * to 1 .. k (and <= 1024 for BF16) -- with launch shapes `tuning_host` (NULL:
 * defaults; timing and use_graph are overridden to 0 and 1), and writes each
 * problem's fastest g to g_host[i] (count entries, caller-owned host
 * memory).  A candidate whose class needs more than workspace_bytes of
 * workspace is skipped; every problem's own g must fit.  The time of the
 * first (dense) iteration is excluded, as in kp_autotune.  Synchronises
 * `stream`; leaves no ctx behind; the workspace contents are undefined
 * afterwards.  KP_ERR_INVALID for invalid problems or tuning, NULL g_host,
 * iters < 2 or a workspace too small for the problems as given. */
kp_status kp_autotune_groups(const kp_problem *problems_host, int32_t count, void *workspace_dev,
                             size_t workspace_bytes, void *stream, int32_t iters, const kp_tuning *tuning_host,
                             int32_t *g_host);

/* ------------------------------------------------------------ diagnostics
 * Two read-only views of what the filtered iteration computes, for tests
 * that check the precision argument directly rather than through the final
 * labels. */

/* The BF16x3 estimate of squared distances exactly as the distance kernels
 * form it, and its error bound (the precision form's derived bound: the
 * distance calculator of Section 1 run on BF16 matrix cores, whose result
 * must still be that of standard K-means, Abstract).  For each of the nq
 * query rows (queries_dev: nq*d FP32, row-major, 16-byte aligned) against
 * every centroid of BF16 problem `problem` (its current FP32 centroids, the
 * initial ones before the first iteration), est_dev[i*k + j] receives the
 * estimate v of ||q_i - c_j||^2 that the decisions compare (the key value,
 * low significand bits cleared) and eta_dev[i*k + j] a bound with
 * |v - ||q_i - c_j||^2| <= eta in exact arithmetic on the FP32 inputs.  j is
 * the original centroid index.  anchor = -1 gives the estimate of the first
 * (dense) iteration and of serving; anchor = a (an original centroid index)
 * gives the form the filtered iterations use for a tile of points sorted to
 * centroid a: every query and centroid taken relative to c_a.  Outputs are
 * caller-owned device buffers of nq*k FP32.  Queued on the ctx's stream.
 * KP_ERR_UNSUPPORTED for an FP32 problem, or an anchor on a problem with more
 * than 16384 centroid slots (which keeps no anchor tables); KP_ERR_INVALID
 * for a bad index or anchor, NULL or misaligned pointers or nq outside
 * 0..2^31-1 (nq = 0 is a no-op). */
kp_status kp_probe_estimates(kp_ctx *ctx, int32_t problem, const float *queries_dev, int64_t nq,
                             int32_t anchor, float *est_dev, float *eta_dev);

/* The bounds the filters of Section 1 keep for the listed points, brought
 * to the current centroids (after the latest update): for each i < np with
 * point x = idx_dev[i] (int32 point index) assigned to centroid a,
 * ub_dev[i] >= d(x, c_a) (the point-level filter's upper bound),
 * lbp_dev[i] <= d(x, c_j) for every j != a (its point-level lower bound) and
 * lb_dev[i*g + q] <= d(x, c_j) for every member j != a of group q (the
 * group-level filter's bounds), in exact arithmetic on the FP32 point and
 * centroids.  group_dev (k int32, may be NULL) receives each original
 * centroid's group.  All outputs are caller-owned device buffers; queued on
 * the ctx's stream.  KP_ERR_STATE before the first iteration; KP_ERR_INVALID
 * for a bad index, NULL outputs or np outside 0..2^31-1.  A listed index
 * outside 0..n-1 is clamped into range. */
kp_status kp_bounds(kp_ctx *ctx, int32_t problem, const int32_t *idx_dev, int64_t np, float *ub_dev,
                    float *lbp_dev, float *lb_dev, int32_t *group_dev);

/* Static description of a status code. */
const char *kp_strerror(kp_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *kp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KP_H */
