/*
 * tnn.h -- exact Trajectory Nearest Neighbours (TNN) on AMD Instinct MI355X.
 *
 * Exact k-nearest-neighbour search over points that lie along time-sorted
 * trajectories, under the per-feature scaled squared metric
 *     d(q, p) = s_x dx^2 + s_y dy^2 + s_z dz^2 + s_t dt^2        (Sec. 3.4)
 * with the strict causal mask  t_p < t_q - t_w                    (Sec. 3.4,
 * masked temporal part; Sec. 3.5).  Trajectories are cut into segments of
 * K consecutive points, each covered by a cylinder (segment plus radius,
 * Sec. 3.4); a query ranks cylinders by a lower bound on the distance to any
 * member, scans the members of the nearest ones and stops once its k-th
 * distance is below every remaining bound (Algorithms 1 and 2).  Results are
 * exactly those of a linear search (Sec. 4.2): ascending (distance, index),
 * distance in binary64 computed as
 *     ((s_x*(dx*dx) + s_y*(dy*dy)) + s_z*(dz*dz)) + s_t*(dt*dt)
 * with dx = (double)q_x - (double)p_x etc., every operation rounded once.
 *
 * Conventions for every entry point:
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary host memory read before the call returns.
 *  - The library never allocates device memory: the caller sizes buffers with
 *    the *_workspace / *_bytes calls and owns them.  Inputs and buffers must
 *    stay alive until the work queued on `stream` (a hipStream_t, NULL = the
 *    default stream) has completed.
 *  - Argument checks run before anything is queued and return a negative
 *    status; nothing is written then.  No C++ exception crosses this ABI.
 *  - Calls that share a scratch buffer must not overlap in time.
 */
#ifndef TNN_H
#define TNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tnn_status;
#define TNN_OK 0
#define TNN_E_ARG (-1)         /* null pointer, bad size, scale < 0 or not finite, k out of range */
#define TNN_E_UNSORTED (-2)    /* a trajectory's times decrease */
#define TNN_E_NONFINITE (-3)   /* a coordinate is NaN or infinite */
#define TNN_E_WORKSPACE (-4)   /* buffer smaller than the size the matching *_workspace call gave */
#define TNN_E_HIP (-5)         /* a HIP runtime call failed */
#define TNN_E_UNSUPPORTED (-6) /* valid request outside the library's limits */
#define TNN_E_FORMAT (-7)      /* a checkpoint that is not a complete, intact checkpoint of
                                  this library's radius model */

/* Structure-of-arrays float32 points in device memory: x, y, z (km), t (s). */
typedef struct {
  const float *x, *y, *z, *t;
  int64_t n;
} tnn_points;

/* Immutable segment index.  Plain data: it only describes device arrays that
 * live in the caller's `d_mem` buffer given to tnn_build_segments, and may be
 * copied freely while that buffer lives. */
typedef struct {
  uint64_t opaque[48];
} tnn_index;

/* Query flags. */
#define TNN_PLAIN 0u       /* TNN, plain: seed from the nearest block, then expand */
#define TNN_BRUTE 1u       /* linear search over every point (Sec. 3.6 baseline) */
#define TNN_MIXED_BF16 2u  /* with TNN_BRUTE: BF16 MFMA distance tiles as a proven
                              lower-bound filter, survivors rescored in binary64.
                              A query whose own scaled squared norm (about the index
                              box centre) reaches 1e30 gets (-1, NaN) slots. */
#define TNN_LEARNED 4u     /* TNN seeded with a predicted k-th distance d_radius2[q] */
#define TNN_LEARNED_SEED 16u /* with TNN_LEARNED: also find the nearest block and scan its
                              seed segments as plain TNN does, then start from the smaller
                              of that k-th distance and the prediction.  Pays when the
                              bounds share a large floor (a time window, Sec. 3.1) and
                              order the blocks poorly; the radius calibration can time
                              both ways and keep the faster.  Results are the same. */

/* Statistics counters (TNN_STAT_*), unsigned 64-bit, accumulated with atomics
 * when tnn_query_params.d_stats is not NULL. */
#define TNN_STAT_QUERIES 0
#define TNN_STAT_BLOCKS 1      /* block lower bounds evaluated */
#define TNN_STAT_SEGMENTS 2    /* segment (cylinder) lower bounds evaluated */
#define TNN_STAT_POINTS 3      /* point distances computed ("comparisons", Sec. 4.2); the BF16
                                  linear search counts the (query, point) pairs of the stages it
                                  scans, its pilot pass's included: a stage whose points all fail
                                  a query tile's time mask is skipped */
#define TNN_STAT_MERGES 4      /* top-k merges */
#define TNN_STAT_ROUNDS 5      /* expansion rounds over all queries */
#define TNN_STAT_FALLBACKS 6   /* learned radius held fewer than k points */
#define TNN_STAT_RESCORED 7    /* binary64 rescoring of filtered candidates (the BF16 linear
                                  search: also its pilot pass's binary64 pairs) */
#define TNN_STAT_MAX_ERR 8     /* bit pattern of the largest |approx - exact| distance (double) */
#define TNN_STAT_COUNT 16

/* Float32 range: TNN's bounds and the BF16 tiles need the scaled squared
 * half-diagonal of the index box, sum_f s_f ((hi_f - lo_f) / 2)^2, below 1e30
 * (TNN_E_UNSUPPORTED otherwise; the binary64 linear search has no limit), and
 * queries within about 1e8 box widths of the data. */
typedef struct {
  double scale[4];          /* s_x, s_y, s_z, s_t >= 0, finite */
  double t_window;          /* t_w >= 0: only points with t < t_q - t_w are candidates */
  int32_t k;                /* 1 .. 64 */
  uint32_t flags;           /* TNN_* flags above */
  int32_t seed_segments;    /* F of Algorithm 2: segments of the nearest block scanned
                               first (1..64; 0 = 4).  TNN only. */
  int32_t waves_per_block;  /* launch shape: 1, 2, 4 or 8 waves of 64 lanes (0 = 4) */
  const float *d_radius2;   /* device [n_queries] predicted k-th distance (metric units,
                               squared).  With TNN_LEARNED exactly one of d_radius2 and
                               radius_model (below) is set; else ignored.  Any value (0,
                               inf, NaN) keeps results exact; it only changes the work
                               done. */
  unsigned long long *d_stats; /* device [TNN_STAT_COUNT] or NULL */
  const double *d_query_scale; /* device [n_queries][4] per-query scales (s_x, s_y, s_z,
                               s_t) replacing `scale` for each query, or NULL (`scale` is
                               still checked: pass any valid values).  The scales
                               may vary over space (Sec. 3.2: sigma as a function of
                               position); the metric of query q is then s_q.  A row with a
                               negative or non-finite entry, or (TNN) out of the float32
                               range above, yields (-1, NaN) in every slot of that query.  TNN (plain or learned) and TNN_BRUTE only:
                               with TNN_MIXED_BF16 or in a tnn_query_batched item it is
                               TNN_E_UNSUPPORTED. */
  /* Optional Gaussian kernel averaging of the neighbours' measurements (Sec.
   * 3.2, Eq. gka; the definition of tnn_gka_average, below): with
   * d_gka_values set, each query's d_gka_out row receives the average of
   * d_gka_values over its k neighbours.  tnn_query runs tnn_gka_average's
   * kernel on the stream right after the search, on the outputs it has just
   * written (on the 1M-point workload this adds less to the call than
   * computing the average inside the search kernel, whose vector units it
   * would share); tnn_query_batched items compute it from the search's
   * registers as soon as a query's neighbours are final.  Results equal
   * tnn_gka_average on the returned idx and dist. */
  const float *d_gka_values;   /* device float32 [n_points][gka_comp], row p = the
                                  measurement at caller point p; NULL = no averaging */
  double *d_gka_out;           /* device binary64 [n_queries][gka_comp]; NaN rows for
                                  queries without context (or without a metric) */
  int32_t gka_comp;            /* components per point, 1..8 (with d_gka_values) */
  /* Radius predicted inside the call: with TNN_LEARNED and radius_model set
   * (and d_radius2 NULL), tnn_query predicts each query's k-th distance
   * (radius_alpha * exp(out))^2 with the model, as tnn_radius_infer does, into
   * its scratch, in the same launch as its per-call preparation; results are
   * those of calling tnn_radius_infer first and passing d_radius2.  Not with
   * TNN_BRUTE or in a tnn_query_batched item (TNN_E_UNSUPPORTED). */
  float radius_alpha;          /* > 0, finite (with radius_model) */
  const void *radius_model;    /* device tnn_radius_model, or NULL */
} tnn_query_params;

/* Human-readable name of a status code (static string). */
const char *tnn_status_string(tnn_status s);

/*
 * Size of the device buffer tnn_build_segments needs.
 * h_traj_offsets: host int64 [n_traj + 1], non-decreasing, offsets[0] = 0;
 * trajectory j holds points offsets[j] .. offsets[j+1]-1.  seg_len = K in 1..64.
 */
tnn_status tnn_build_segments_workspace(const int64_t *h_traj_offsets, int64_t n_traj,
                                        int32_t seg_len, size_t *bytes);

/*
 * Build the segment index (Sec. 3.4, partition and segment approximation).
 * Each trajectory is cut into runs of seg_len consecutive points (the last run
 * may be shorter; no padding copies).  A run becomes a segment from its first
 * point A to its last point B with t_min / t_max and a per-axis approximation
 * error e_f = max |P_f - Q_f| over members P, Q the clamped Euclidean
 * projection of P on AB, computed in binary64 and rounded up to float32.
 * Segments are reordered into spatially compact blocks of 64 (recursive median
 * split along the widest axis scaled by sqrt(order_scale), split points on
 * multiples of 64, ties by segment number, each part keeping its order; inside
 * a block the halving goes on down to single segments; made on the device;
 * NULL keeps trajectory order), points are copied in segment order, and each
 * block gets the bounding box of its points.
 * pts: device SoA, trajectory-contiguous, times non-decreasing within each
 * trajectory (else TNN_E_UNSORTED), finite (else TNN_E_NONFINITE).
 * order_scale: host double[4] or NULL.  d_mem/bytes: device buffer of at least
 * tnn_build_segments_workspace bytes; it holds the index afterwards.
 * Synchronous: returns after the work on `stream` has finished.
 */
tnn_status tnn_build_segments(tnn_points pts, const int64_t *h_traj_offsets, int64_t n_traj,
                              int32_t seg_len, const double *order_scale, void *d_mem,
                              size_t bytes, void *stream, tnn_index *out);

/* Sizes of a built index (any output pointer may be NULL). */
tnn_status tnn_index_info(const tnn_index *index, int64_t *n_points, int64_t *n_segments,
                          int64_t *n_blocks, int32_t *seg_len);

/* Scratch bytes tnn_query needs for n_queries queries with these params.
 * TNN: the per-call segment records (constants that depend on the scales)
 * and the counters of the search's work queues (and 4 B per query for the
 * predicted radius when params->radius_model is set).  TNN_BRUTE: none (256).
 * TNN_BRUTE | TNN_MIXED_BF16: the BF16 point operands (64 B per point,
 * padded to 128 points), |v|^2 per point, each query's top-k lists (12 B per
 * slot: one list per point chunk, 1 to 16 chunks chosen from n_queries and
 * the point count, plus the pilot pass's), its bound, home block and place
 * in the scan order, per-block query counts, the tiles' first stages, each
 * stage's earliest time, and a work counter.  tnn_query writes all of it
 * itself, so the buffer needs no initialisation, but two calls in flight at
 * once must not share it. */
tnn_status tnn_query_workspace(const tnn_index *index, int64_t n_queries,
                               const tnn_query_params *params, size_t *bytes);

/*
 * k-NN of every query (Algorithms 1 and 2).  For query q, writes
 * d_out_idx[q*k + r] (int32, caller's point index) and d_out_dist[q*k + r]
 * (binary64 scaled squared distance), r = 0..k-1 ascending by (distance,
 * index); empty slots are (-1, +inf).  A zero distance is reported as +0.0
 * (scales of -0.0 would otherwise give -0.0, which equals it).  Queries are
 * device SoA float32 and need not be data points.  Asynchronous on `stream`.
 */
tnn_status tnn_query(const tnn_index *index, tnn_points queries, const tnn_query_params *params,
                     int32_t *d_out_idx, double *d_out_dist, void *d_scratch,
                     size_t scratch_bytes, void *stream);

/*
 * tnn_query without a scratch argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and flags as tnn_query;
 * the scratch it needs is a library-owned device array of
 * TNN_NOALLOC_SCRATCH_BYTES per GPU (one copy on each device the library runs
 * on, kept until the process ends), so calls whose tnn_query_workspace size
 * exceeds it return TNN_E_WORKSPACE before anything is queued (TNN: about
 * 64 B per segment, so indexes of up to about 262k segments, 8M points at
 * K = 32).  The array is resolved once per device on that device's first
 * call.  Nothing is allocated: no hipMalloc, no hipFree.  Every call on a
 * device shares that device's array: two calls that overlap in time on one
 * device (two streams, two threads) race and must not be issued.  Asynchronous
 * on `stream`.
 */
#define TNN_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
tnn_status tnn_query_noalloc(const tnn_index *index, tnn_points queries,
                             const tnn_query_params *params, int32_t *d_out_idx,
                             double *d_out_dist, void *stream);

/*
 * Test export of the index: per segment in index order
 * d_seg_f32[12*s + 0..11] = A.xyz, B.xyz, t_min, t_max, e.xyz, 0;
 * d_seg_i32[4*s + 0..3] = trajectory-order segment number, first point slot in
 * index order, member count, block; d_point_id[i] = caller index of the point
 * stored at slot i; d_block_box[8*b + 0..7] = lo.xyzt, hi.xyzt.
 * Any output may be NULL.  Asynchronous.
 */
tnn_status tnn_debug_export_index(const tnn_index *index, float *d_seg_f32, int32_t *d_seg_i32,
                                  int32_t *d_point_id, float *d_block_box, void *stream);

/*
 * Test export of the bounds the query kernels use: d_seg_lb[q*S + s]
 * (binary64, segment s in index order) and d_block_lb[q*nb + b] (float32);
 * +inf where masked.  Either output may be NULL.  h_scale: the shared scales.
 * d_query_scale: device [n_queries][4] per-query scales or NULL; with it each
 * query's cylinder bounds are the ones the per-query-scale search forms for
 * its own metric, and a row the search would refuse (a negative or
 * non-finite scale, or out of the float32 range) gets NaN bounds.
 * Asynchronous.
 */
tnn_status tnn_debug_lower_bounds(const tnn_index *index, tnn_points queries,
                                  const double *h_scale, double t_window,
                                  const double *d_query_scale, double *d_seg_lb,
                                  float *d_block_lb, void *d_scratch, size_t scratch_bytes,
                                  void *stream);


/* ------------------------------------------------------------------------
 * Learned k-th radius (not in the paper): a 6-64-64-1 ReLU MLP predicting
 * log r_k, r_k = sqrt(d_k) the k-th neighbour's distance, from the query's
 * coordinates mapped to [-1, 1] over the data's bounding box,
 * 0.25*log1p(segment count of its cell in a 32^3 (x, y, t) grid), and
 * 0.5*log1p(trajectory starts in its cell of a finer 128 x 128 x 512 grid,
 * the 8 spatial neighbours, and those 9 cells one time step earlier; cells
 * outside the grid add nothing).  Its prediction seeds TNN_LEARNED queries;
 * results stay exact whatever it says.
 * ------------------------------------------------------------------------ */
#define TNN_RADIUS_HIDDEN 64
#define TNN_RADIUS_INPUTS 6
#define TNN_RADIUS_GRID 32
#define TNN_RADIUS_START_XY 128
#define TNN_RADIUS_START_T 512
#define TNN_RADIUS_NPARAMS (TNN_RADIUS_HIDDEN * TNN_RADIUS_INPUTS + TNN_RADIUS_HIDDEN + \
                            TNN_RADIUS_HIDDEN * TNN_RADIUS_HIDDEN + TNN_RADIUS_HIDDEN +     \
                            TNN_RADIUS_HIDDEN + 1)

/* Device layout of a radius model (the payload of a checkpoint, below). */
typedef struct {
  float params[TNN_RADIUS_NPARAMS]; /* W1[64][6] b1[64] W2[64][64] b2[64] W3[64] b3 */
  float pad[3];
  float lo[4], hi[4];               /* bounding box of the indexed points (x, y, z, t) */
  int32_t grid[TNN_RADIUS_GRID * TNN_RADIUS_GRID * TNN_RADIUS_GRID]; /* [x][y][t] */
  /* per cell [x][y][t]: trajectories whose first point falls in the cell, its
   * 8 spatial neighbours, or those 9 cells one time step earlier (saturating) */
  uint16_t starts[TNN_RADIUS_START_XY * TNN_RADIUS_START_XY * TNN_RADIUS_START_T];
} tnn_radius_model;

/* sizeof(tnn_radius_model). */
tnn_status tnn_radius_model_bytes(size_t *bytes);

/* Fill a model for `index`: bounding box and density grid from the index,
 * weights drawn uniformly in +-sqrt(6 / fan_in) from a counter-based hash of
 * `seed` (biases 0).  d_model: device, tnn_radius_model_bytes.  Async. */
tnn_status tnn_radius_model_init(const tnn_index *index, void *d_model, uint64_t seed,
                                 void *stream);

/* Scratch bytes of tnn_radius_grad / tnn_radius_train_step for `batch`. */
tnn_status tnn_radius_train_workspace(int64_t batch, size_t *bytes);

/*
 * Training order for one epoch: d_order[i] (device int32 [n]) receives a
 * permutation of 0 .. n-1 drawn from `seed` (a keyed 4-round Feistel
 * permutation of [0, 4^h), 4^h >= n, walked along its cycles until it lands
 * below n; SplitMix64 round function).  The same seed gives the same order.
 * Async.  TNN_E_ARG for n < 0, n > INT32_MAX or a null d_order with n > 0.
 */
tnn_status tnn_radius_shuffle(int64_t n, uint64_t seed, int32_t *d_order, void *stream);

/*
 * Gradient of the mean squared error between the MLP output and the label
 * log(sqrt(d)) over the batch b = 0 .. batch-1 of samples i = d_order[first + b]
 * (or first + b when d_order is NULL), where d = d_dist[i*k + k-1] (the k-th
 * distance tnn_query wrote for sample i); samples whose d is not finite and
 * positive are left out.  Writes d_grad[NPARAMS] (float32, device) and
 * *d_loss (float32, device; may be NULL).  Sums run in a fixed order: the
 * result is deterministic.  Async.
 */
tnn_status tnn_radius_grad(const void *d_model, tnn_points samples, const double *d_dist,
                           const int32_t *d_order, int32_t k, int64_t first, int64_t batch,
                           float *d_grad, float *d_loss, void *d_scratch, size_t scratch_bytes,
                           void *stream);

/*
 * One Adam step (Kingma & Ba 2015, beta1 0.9, beta2 0.999, eps 1e-8) on that
 * gradient.  d_adam: device float[2*NPARAMS] (first and second moments),
 * zero before step 1; `step` counts from 1.  Async.
 */
tnn_status tnn_radius_train_step(void *d_model, float *d_adam, tnn_points samples,
                                 const double *d_dist, const int32_t *d_order, int32_t k,
                                 int64_t first, int64_t batch, int32_t step, float lr,
                                 float *d_loss, void *d_scratch, size_t scratch_bytes,
                                 void *stream);

/* Scratch bytes of tnn_radius_calibrate for n_samples samples. */
tnn_status tnn_radius_calibrate_workspace(int64_t n_samples, size_t *bytes);

/*
 * Safety factor of the predicted radius: *d_alpha (device float32) =
 * exp(x_q) with x_q the q-quantile (linear interpolation between the order
 * statistics at position (m - 1) q, q in [0, 1]) of the binary64
 * log-residuals 0.5 log d_i - out_i over the m samples whose k-th distance
 * d_i = d_dist[i*k + k-1] is finite and positive and whose residual is
 * finite; out_i is the model's output for sample i.  About (1 - q) of such
 * samples then lie outside the radius alpha exp(out).  m = 0 gives 1.  Async.
 */
tnn_status tnn_radius_calibrate(const void *d_model, tnn_points samples, const double *d_dist,
                                int32_t k, double quantile, float *d_alpha, void *d_scratch,
                                size_t scratch_bytes, void *stream);

/*
 * Checkpoint of a radius model: a 64-byte header (magic "TNNRADM", format
 * version 1, payload size, the model's dimensions: hidden units, inputs,
 * grid sizes, parameter count; FNV-1a 64 checksum of the payload) followed
 * by the model's bytes.  tnn_radius_checkpoint_bytes gives the size;
 * tnn_radius_model_save writes it to host memory h_buf (at least that many
 * bytes) and tnn_radius_model_load reads one back into a device model,
 * returning TNN_E_FORMAT for a buffer that is not exactly a complete, intact
 * checkpoint of this version and these dimensions.  Both are synchronous.
 */
tnn_status tnn_radius_checkpoint_bytes(size_t *bytes);
tnn_status tnn_radius_model_save(const void *d_model, void *h_buf, size_t bytes, void *stream);
tnn_status tnn_radius_model_load(const void *h_buf, size_t bytes, void *d_model, void *stream);

/* Test export: the 5 features of each query, d_feat[5*i + j].  Async. */
tnn_status tnn_radius_features(const void *d_model, tnn_points queries, float *d_feat,
                               void *stream);

/*
 * Predicted k-th distance per query: d_radius2[i] = (alpha * exp(out_i))^2,
 * float32 (the TNN_LEARNED seed); d_logr (nullable) receives out_i.  Async.
 */
tnn_status tnn_radius_infer(const void *d_model, tnn_points queries, float alpha,
                            float *d_radius2, float *d_logr, void *stream);

/* ------------------------------------------------------------------------
 * Batched ragged serving: many independent indexes ("airspaces"), each with
 * its own queries, k, scales and flags, answered by one persistent launch.
 * Waves pull chunks of queries from a device work counter, heaviest airspace
 * first (longest-processing-time order by estimated cost), so a whole batch
 * is one kernel and can be captured in a HIP graph and replayed.
 * ------------------------------------------------------------------------ */
typedef struct {
  const tnn_index *index;   /* host pointer to a built index */
  tnn_points queries;       /* device SoA */
  tnn_query_params params;  /* TNN_PLAIN or TNN_LEARNED only; k 1..64 */
  int32_t *d_out_idx;       /* device [queries.n * k] */
  double *d_out_dist;       /* device [queries.n * k] */
} tnn_batch_item;

/* Launch shape of the persistent kernel (0 fields = defaults). */
typedef struct {
  int32_t chunk;            /* queries per pull from the work counter (1..64; 0 = 8) */
  int32_t waves_per_block;  /* 1, 2, 4 or 8 (0 = 4) */
  int32_t blocks_per_cu;    /* resident workgroups per compute unit (1..16; 0 = 4) */
  int32_t reserved;
} tnn_batch_config;

/* Plan of a prepared batch: plain data describing device buffers that live in
 * the scratch given to tnn_batch_prepare. */
typedef struct {
  uint64_t opaque[16];
} tnn_batch_plan;

#define TNN_MAX_BATCH_ITEMS 1024

/* Scratch bytes of tnn_batch_prepare for these items (1..TNN_MAX_BATCH_ITEMS). */
tnn_status tnn_batch_workspace(const tnn_batch_item *items, int32_t n_items, size_t *bytes);

/*
 * Validate the items, order them by estimated cost and upload the descriptor
 * table into d_scratch (synchronous: not for graph capture).  The items'
 * buffers must outlive every tnn_query_batched call on the plan.
 */
tnn_status tnn_batch_prepare(const tnn_batch_item *items, int32_t n_items,
                             const tnn_batch_config *config, void *d_scratch, size_t bytes,
                             void *stream, tnn_batch_plan *plan);

/*
 * Answer every item's queries (same results as one tnn_query per item).
 * Queues only kernels (per-item preparation, a counter reset, the persistent
 * search): safe inside HIP graph capture and replay.  Also records device
 * wall-clock ticks: ticks[0] at the start, ticks[1 + i] when item i's last
 * query is written (see tnn_batch_ticks, tnn_wall_clock_rate_khz).  Async.
 */
tnn_status tnn_query_batched(const tnn_batch_plan *plan, void *stream);

/* Device pointer to the plan's uint64 tick array [n_items + 1]. */
tnn_status tnn_batch_ticks(const tnn_batch_plan *plan, const uint64_t **d_ticks);

/* Frequency of the device wall clock used for the ticks, in kHz. */
tnn_status tnn_wall_clock_rate_khz(int64_t *khz);

/*
 * Autotuner: times the candidate launch shapes of the persistent kernel on
 * these items (each candidate prepared and run on `stream`) and returns the
 * fastest in *best.  With cache_path (nullable) the choice is read from / added
 * to a small text cache keyed by device, item count, total queries and points,
 * so later runs skip the search.  Synchronous.
 */
tnn_status tnn_autotune_batched(const tnn_batch_item *items, int32_t n_items, void *d_scratch,
                                size_t bytes, void *stream, const char *cache_path,
                                tnn_batch_config *best);

/* ------------------------------------------------------------------------
 * Gaussian kernel averaging over the k-NN context (Sec. 3.2, Eq. gka): the
 * forecast at each query is sum_c w_c v_c / sum_c w_c over its context slots
 * c (the k neighbours tnn_query returned, slots with index -1 skipped), with
 * w_c = exp(-d_c) and d_c the returned scaled squared distance, i.e. the
 * kernel's (sigma_xy, sigma_xy, sigma_z, sigma_t) are the search scales.  The
 * printed exponent has no minus sign; only a decaying kernel weights nearer
 * measurements more.  Weights are computed relative to the nearest slot,
 * exp(-(d_c - d_0)), which leaves the ratio unchanged and avoids 0/0 for far
 * contexts.  Binary64 throughout.
 * ------------------------------------------------------------------------ */

/*
 * d_idx, d_dist: device [n_queries * k], as tnn_query wrote them.
 * d_values: device float32 [n_points * n_comp], row p = the measurement at
 * caller point p (n_comp 1..8 components, e.g. a wind vector).
 * d_out: device binary64 [n_queries * n_comp]; NaN rows for queries without
 * context.  Indices outside [0, n_points) count as empty slots.  Async; no
 * scratch.  Errors: TNN_E_ARG for null pointers (with n_queries > 0), k outside
 * 1..64, n_comp outside 1..8, negative sizes.
 */
tnn_status tnn_gka_average(const int32_t *d_idx, const double *d_dist, int64_t n_queries,
                           int32_t k, const float *d_values, int32_t n_comp, int64_t n_points,
                           double *d_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TNN_H */
