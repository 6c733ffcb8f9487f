/*
 * raster.h -- C ABI of the MI355X (gfx950) RASTER library.
 *
 * RASTER ("Contraction Clustering", Ulm et al.) clusters 2-D points in two
 * steps (Algorithm 1):
 *   contraction   -- project every point onto an integer tile by scaling by
 *                    10^p and truncating (Section 3.2), count the points per
 *                    tile, keep the tiles holding at least tau points;
 *   agglomeration -- join significant tiles that touch (Chebyshev distance 1,
 *                    all eight neighbours, Section 3.2) into clusters and keep
 *                    the clusters of at least mu tiles.
 * The input may be cut into chunks fed in any order without changing the
 * result (Section 3.6), which the streaming calls below expose.
 *
 * Conventions shared by every call:
 *   - Points are caller-owned DEVICE memory, row-major (n, 2): x then y of
 *     each point, RASTER_F64 (16 bytes per point, 16-byte aligned) or
 *     RASTER_F32 (8 bytes per point, 8-byte aligned); (n, 3) with
 *     raster_options.dims = 3 (three-dimensional points, below).  FP32 coordinates are
 *     widened to FP64 exactly before the product, so an FP32 point and its
 *     FP64 widening land on the same tile.
 *   - Tile of a point: kx = trunc(fl64(x * s)), ky = trunc(fl64(y * s)), one
 *     IEEE binary64 product rounded to nearest, truncated toward zero.  With an
 *     integer precision p in [0, 15], s = 10^p exactly.  A coordinate whose
 *     product is not finite or has magnitude >= 2^31 - 1 makes the whole call
 *     fail with RASTER_E_RANGE.
 *   - Tile key: the 64-bit "biased key" (uint64)(kx + 2^31) << 32 |
 *     (uint32)(ky + 2^31).  Unsigned order of keys is lexicographic (kx, ky)
 *     order.  A cluster's label is the smallest key among its tiles.
 *   - Significant means count >= tau (tau >= 1).  A cluster is kept when it
 *     holds at least mu tiles (mu >= 1).
 *   - Every call returns a raster_status; 0 is success.  On failure no
 *     result is produced (*out stays NULL) and raster_last_error() gives a
 *     one-line reason for the calling thread.
 *   - Work is enqueued on the caller's HIP stream (0 = the null stream).  Calls
 *     that return a result synchronise that stream, because output sizes depend
 *     on the data.
 *   - The library allocates its own device memory (tables, scratch, results);
 *     results are owned by the library until raster_result_free().
 */
#ifndef RASTER_H
#define RASTER_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum raster_dtype { RASTER_F32 = 1, RASTER_F64 = 2 } raster_dtype;

/* Distance in the neighbourhood of a tile (Section 3.2 allows a Chebyshev or
 * a Manhattan distance of delta steps; the paper's code, and every call
 * without a _delta suffix, uses Chebyshev 1: the eight adjacent tiles). */
typedef enum raster_metric { RASTER_CHEBYSHEV = 0, RASTER_MANHATTAN = 1 } raster_metric;
#define RASTER_MAX_DELTA 8

/* Variants of the method, for raster_cluster_opts and raster_begin_opts (and,
 * without dims = 3, per job in raster_cluster_batch_opts and
 * raster_server_submit_opts).
 * NULL options mean {RASTER_CHEBYSHEV, 1, 0, 2}: Algorithm 1 as the paper's
 * code runs it. */
typedef struct raster_options {
    raster_metric metric;  /* neighbourhood metric (Section 3.2)                      */
    uint32_t delta;        /* neighbourhood distance, 1 .. RASTER_MAX_DELTA            */
    uint32_t square_step;  /* 1: the 2x2 post-step of Section 3.6 (below), else 0      */
    uint32_t dims;         /* 2 (or 0): points (n, 2); 3: points (n, 3), Section 3.6's
                              generalisation to three dimensions (below)              */
} raster_options;

typedef enum raster_status {
    RASTER_OK = 0,
    RASTER_E_INVAL = -1,  /* bad argument: tau or mu 0, NULL pointer with n > 0,
                             unknown dtype, misaligned points, precision outside
                             [0, 15], non-finite or non-positive scale        */
    RASTER_E_RANGE = -2,  /* a coordinate is NaN/Inf or its tile is out of range,
                             or more than 2^32 - 1 points went into one table */
    RASTER_E_NOMEM = -3,  /* device allocation failed, or a table would need
                             more than 2^31 slots (about 1.29G distinct tiles
                             at the default load factor; 0.97G in three
                             dimensions, whose tables are kept emptier)       */
    RASTER_E_DEVICE = -4, /* a HIP call failed                                 */
    RASTER_E_STATE = -5,  /* streaming call in the wrong state                 */
    RASTER_E_BUDGET = -6  /* server: a single job exceeds the memory budget    */
} raster_status;

typedef struct raster_result raster_result; /* opaque; arrays live on the device */
typedef struct raster_stream raster_stream; /* opaque streaming state; owns the tile table */
typedef struct raster_server raster_server; /* opaque serving loop */

/* Counters and per-phase device times of one clustering run. */
typedef struct raster_stats {
    int64_t n_points;          /* points counted                                  */
    int64_t distinct_tiles;    /* m: tiles holding at least one point             */
    int64_t significant_tiles; /* s: tiles holding at least tau points            */
    int64_t components;        /* connected components of the significant tiles   */
    int64_t clusters;          /* components with at least mu tiles               */
    int64_t tiles;             /* tiles of the kept clusters (rows of the result) */
    int64_t table_capacity;    /* slots of the device tile table                  */
    int64_t grow_events;       /* times the table was enlarged and rehashed       */
    float us_contract;         /* projection + counting (all chunks), microseconds */
    float us_threshold;        /* significance scan and compaction                */
    float us_agglomerate;      /* neighbour union-find                            */
    float us_filter;           /* mu filter, labels and output compaction         */
    int64_t count_launches;    /* launches of the kernel that streams the points   */
    float us_count_kernel;     /* their summed device time, microseconds          */
    float us_bin_keys;         /* binned path: second-level binning, summed       */
    float us_aggregate;        /* binned path: LDS partition updates, summed      */
    int32_t flushes;           /* binned path: groups of keys applied to the table */
    int32_t redone;            /* batched and served jobs: 1 when the job overflowed its
                                  batch table and was redone alone by the plain path */
    int32_t key_frame;         /* 1 when the table placed keys by a key frame and the
                                  binned contraction moved 4-byte entries         */
    int32_t reserved_;         /* 0                                                */
} raster_stats;

/* Launch knobs of the contraction kernels.  Any value gives the same result;
 * they trade speed only.  raster_set_tuning(NULL) restores the defaults. */
typedef struct raster_tuning {
    int32_t block;        /* threads per workgroup of the counting kernel: 64..1024, multiple of 64 */
    int32_t items;        /* points per thread per sweep: 1..16                                   */
    int32_t preagg_slots; /* LDS pre-aggregation slots per workgroup (0 = off, else power of two
                             in [256, 4096]): duplicate tiles within a workgroup's points are
                             combined in LDS before touching the device table               */
    float load_factor;    /* target occupancy of the device table in (0.05, 0.9]               */
    int32_t mode;         /* counting path: 0 auto, 1 direct (one device atomic per point),
                             2 binned (keys binned by table partition, then each partition
                             updated in LDS by one workgroup; used when the table has
                             128..65536 partitions of 4096 slots, else direct), 3 binned
                             with 8-byte bin entries only (2 and 0 move 4-byte entries
                             when a sample of the first chunk shows the tiles of a
                             two-dimensional input within a window of 2^20 x 2^20)     */
    int32_t group_mpoints; /* binned path: millions of points binned before the table is
                              updated (1..4096); bounds the binning and spill buffers      */
} raster_tuning;

/* ---- plain form (Algorithm 1 on one resident point set) -------------------- */

/* Cluster n points with integer precision p in [0, 15] (tile side 10^-p).
 * d_points: device pointer, borrowed until the call returns.  n may be 0. */
raster_status raster_cluster(const void* d_points, int64_t n, raster_dtype dt, int32_t precision,
                             uint32_t tau, uint32_t mu, hipStream_t stream, raster_result** out);

/* Same with an arbitrary positive finite scale s (tile side 1/s), e.g.
 * s = 10^3.5 for the paper's non-integer precisions (Section 3.2). */
raster_status raster_cluster_scaled(const void* d_points, int64_t n, raster_dtype dt, double scale,
                                    uint32_t tau, uint32_t mu, hipStream_t stream,
                                    raster_result** out);

/* Same with a wider or Manhattan neighbourhood: two significant tiles belong
 * to one cluster when a chain of significant tiles joins them in which each
 * step is at most `delta` tiles in `metric` (Section 3.2, Algorithm 1's
 * neighbors(u, delta)).  1 <= delta <= RASTER_MAX_DELTA, else E_INVAL.  The
 * agglomeration makes one pass over the table per four backward offsets of
 * the neighbourhood (Chebyshev delta has 2 delta (delta + 1) of them,
 * Manhattan delta has delta (delta + 1)). */
raster_status raster_cluster_delta(const void* d_points, int64_t n, raster_dtype dt, double scale,
                                   uint32_t tau, uint32_t mu, raster_metric metric, uint32_t delta,
                                   hipStream_t stream, raster_result** out);

/* Same with every variant in `opts` (NULL: the defaults).  dims = 3 takes
 * three-dimensional points, row-major (n, 3) (8-byte aligned for FP64, 4 for
 * FP32): each coordinate is projected as in two dimensions, tiles must satisfy
 * |k| <= 2^20 - 2 (else E_RANGE), and the neighbourhood ranges over all three
 * coordinates (Chebyshev 1: the 26 surrounding tiles; Manhattan 1: the 6 face
 * neighbours).  The label is the biased key of the cluster's smallest tile in
 * (x, y, z) order, ((kx + 2^20) << 42) | ((ky + 2^20) << 21) | (kz + 2^20);
 * the third coordinate of each row comes from raster_result_kz.  Not with
 * square_step or in batches.  square_step = 1
 * adds the post-step that Section 3.6 proposes for points spread over the
 * tiles around a grid corner (Figure 4): a tile with fewer than tau points is
 * also significant when some 2x2 square of tiles containing it holds at least
 * tau points together (counted before any tile is dropped).  Only tiles with
 * points are retained.  It adds one pass over the table that probes the eight
 * surrounding tiles of every tile below tau.  E_INVAL for an unknown metric,
 * delta outside [1, RASTER_MAX_DELTA], square_step not 0 or 1, or dims not 0,
 * 2 or 3. */
raster_status raster_cluster_opts(const void* d_points, int64_t n, raster_dtype dt, double scale,
                                  uint32_t tau, uint32_t mu, const raster_options* opts, hipStream_t stream,
                                  raster_result** out);

/* raster_cluster_opts with an integer precision p in [0, 15] (s = 10^p,
 * computed exactly by the library) instead of a scale; E_INVAL for p outside
 * [0, 15]. */
raster_status raster_cluster_p_opts(const void* d_points, int64_t n, raster_dtype dt, int32_t precision,
                                    uint32_t tau, uint32_t mu, const raster_options* opts, hipStream_t stream,
                                    raster_result** out);

/* ---- plain form without device allocation ------------------------------------ */

/* For callers that cannot allocate device memory: code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * raster_cluster (precision p in [0, 15], Chebyshev 1, two dimensions) on at
 * most RASTER_NOALLOC_MAX_POINTS points, with every scratch buffer (tile
 * table, compact arrays, union-find words, counters) in one fixed device
 * array of RASTER_NOALLOC_SCRATCH_BYTES that the library holds on each device
 * it runs on until the process ends; the call itself allocates nothing.
 * The kept rows are written to the caller's device arrays d_kx, d_ky (int32),
 * d_count (uint32) and d_label (uint64, the biased key of the cluster's
 * smallest tile), each of at least max_rows elements, in no particular
 * order; *rows (host) receives the number of rows t.  The rows, as a set,
 * are those of raster_cluster on the same points.  stats, if not NULL,
 * receives the counters (the phase times are 0).  Synchronises `stream`.
 * Errors: E_INVAL for the argument errors of raster_cluster, for n above
 * RASTER_NOALLOC_MAX_POINTS, for rows NULL, and when t > max_rows (then *rows
 * is t and no row is written: max_rows = n always suffices); E_RANGE as for
 * raster_cluster; E_NOMEM if the fixed table (at least four slots per point)
 * overflows, which takes an adversarial point set.
 * The array is shared by every call on the device and keeps the last call's
 * contents; each call clears what must start empty.  Calls on one device are
 * serialised by the library (a call holds the device's array until it has
 * synchronised its stream); calls from another process use that process's
 * own array. */
#define RASTER_NOALLOC_MAX_POINTS (1 << 19)
#define RASTER_NOALLOC_SCRATCH_BYTES 52634368u
raster_status raster_cluster_noalloc(const void* d_points, int64_t n, raster_dtype dt, int32_t precision,
                                     uint32_t tau, uint32_t mu, hipStream_t stream, int32_t* d_kx,
                                     int32_t* d_ky, uint32_t* d_count, uint64_t* d_label, int64_t max_rows,
                                     int64_t* rows, raster_stats* stats);

/* ---- results --------------------------------------------------------------- */

int64_t raster_result_num_tiles(const raster_result* r);    /* rows t, or -1 if r is NULL */
int64_t raster_result_num_clusters(const raster_result* r); /* kept clusters, or -1      */
/* Borrowed device arrays of t rows each: tile kx, ky, its point count and its
 * cluster label (biased key of the cluster's smallest tile).  Rows are in no
 * particular order; any NULL out-pointer is skipped.  Valid until the free. */
raster_status raster_result_arrays(const raster_result* r, const int32_t** d_kx,
                                   const int32_t** d_ky, const uint32_t** d_count,
                                   const uint64_t** d_label);
/* Copy the t rows into caller-owned device buffers (each of at least t
 * elements; NULL skips an array), enqueued on `stream` without waiting. */
raster_status raster_result_copy(const raster_result* r, int32_t* d_kx, int32_t* d_ky, uint32_t* d_count,
                                 uint64_t* d_label, hipStream_t stream);
raster_status raster_result_stats(const raster_result* r, raster_stats* out);
/* The third tile coordinate of every row of a three-dimensional result
 * (borrowed device array of t int32, valid until raster_result_free); NULL for
 * a two-dimensional result. */
raster_status raster_result_kz(const raster_result* r, const int32_t** d_kz);
/* Copy the t third coordinates of a three-dimensional result into a
 * caller-owned device array of at least t int32, enqueued on `stream`; E_INVAL
 * for a two-dimensional result. */
raster_status raster_result_copy_kz(const raster_result* r, int32_t* d_kz, hipStream_t stream);
void raster_result_free(raster_result* r);

/* Per-point labels: the label of every input point, obtained as in the
 * paper's comparison experiment (Section 4.1, its RASTER-star variant) by
 * projecting the points a second time.  Each of the n points of d_points
 * ((n, 2) row-major, or (n, 3) for a three-dimensional result; dt as for
 * clustering, borrowed for the call) is projected
 * with the scale the result was computed with; d_labels[i] (caller-owned
 * device array of n uint64, 8-byte aligned) receives the label of the kept
 * cluster its tile belongs to (the biased key of that cluster's smallest
 * tile, as in the rows), or 0xFFFFFFFFFFFFFFFF (-1 as int64) when its tile is
 * in no kept cluster.  The points need not be the ones that were clustered.
 * The first call builds a device lookup table of the result's tiles, kept
 * with the result until raster_result_free.  Synchronises `stream`.  Errors:
 * E_INVAL for bad arguments; E_RANGE if a point is not finite or its tile is
 * outside +-(2^31 - 2) (+-(2^20 - 2) in three dimensions; that point's label
 * is then -1; the others are written).  Calls on one result are serialised. */
raster_status raster_result_point_labels(raster_result* r, const void* d_points, int64_t n, raster_dtype dt,
                                         uint64_t* d_labels, hipStream_t stream);

/* Per-tile point lists (RASTER', Section 3.4): the points of every kept tile.
 * The paper's RASTER' keeps each tile's points in the hash table during
 * contraction; here they are gathered after clustering by projecting the
 * points a second time, which gives the same sets.  For the n points of
 * d_points ((n, 2), or (n, 3) for a three-dimensional result; borrowed for
 * the call; n < 2^32 - 1), the indices of the points
 * on row j of the result (the row order of raster_result_arrays) are
 * d_index[d_row_start[j] .. d_row_start[j + 1]), in no particular order within
 * a row.  d_row_start: caller-owned device array of t + 1 uint64;
 * d_index: caller-owned device array of `cap` uint64 (cap >= the number of
 * points on kept tiles; n always suffices).  *n_kept (host) receives that
 * number.  Points on no kept tile are not listed.  Synchronises `stream`.
 * Errors: E_INVAL for bad arguments, or when cap is too small (then
 * d_row_start and *n_kept are written, d_index is not); E_RANGE if a point is
 * not finite or its tile is outside +-(2^31 - 2) (+-(2^20 - 2) in three
 * dimensions).  Calls on one result are serialised. */
raster_status raster_result_tile_points(raster_result* r, const void* d_points, int64_t n, raster_dtype dt,
                                        uint64_t* d_row_start, uint64_t* d_index, int64_t cap, int64_t* n_kept,
                                        hipStream_t stream);

/* ---- streaming form (chunked input, Section 3.6) ---------------------------- */

/* Start a stream.  tile_hint: expected number of distinct tiles (0 = unknown);
 * the table grows by rehashing when it fills, so the hint only saves time.
 * The stream owns one device tile table for its whole life (constant memory). */
raster_status raster_begin(int32_t precision, uint32_t tau, uint32_t mu, int64_t tile_hint,
                           hipStream_t stream, raster_stream** st);
raster_status raster_begin_scaled(double scale, uint32_t tau, uint32_t mu, int64_t tile_hint,
                                  hipStream_t stream, raster_stream** st);
/* A stream whose agglomeration uses the neighbourhood (metric, delta), as in
 * raster_cluster_delta. */
raster_status raster_begin_delta(double scale, uint32_t tau, uint32_t mu, raster_metric metric, uint32_t delta,
                                 int64_t tile_hint, hipStream_t stream, raster_stream** st);
/* A stream with every variant in `opts`, as in raster_cluster_opts. */
raster_status raster_begin_opts(double scale, uint32_t tau, uint32_t mu, const raster_options* opts,
                                int64_t tile_hint, hipStream_t stream, raster_stream** st);
/* raster_begin_opts with an integer precision p in [0, 15] (s = 10^p), as in
 * raster_begin. */
raster_status raster_begin_p_opts(int32_t precision, uint32_t tau, uint32_t mu, const raster_options* opts,
                                  int64_t tile_hint, hipStream_t stream, raster_stream** st);
/* Count one chunk.  d_points is borrowed until the stream has passed the
 * enqueued work (the next raster_* call on this stream object, or a
 * synchronisation of its HIP stream).  Returns without waiting for this chunk;
 * it may wait for the previous chunk's counters to decide whether the table
 * must grow.  A range error moves the stream to a failed state, reported by
 * this or a later call; every later call then returns RASTER_E_STATE or the
 * recorded error. */
raster_status raster_feed_chunk(raster_stream* st, const void* d_points, int64_t n,
                                raster_dtype dt);
/* Significance filter and agglomeration over everything fed so far.  The
 * stream is finished afterwards: further feeds return RASTER_E_STATE. */
raster_status raster_finish(raster_stream* st, raster_result** out);
/* Tiles counted so far (before the tau filter), for checking the contraction.
 * Writes up to cap (key, count) pairs into caller device buffers and the true
 * number of tiles into *m; synchronises the stream. */
raster_status raster_stream_tiles(raster_stream* st, uint64_t* d_keys, uint32_t* d_counts,
                                  int64_t cap, int64_t* m);
/* Free the stream and its table; allowed in any state. */
void raster_stream_destroy(raster_stream* st);

/* ---- batched form ------------------------------------------------------------ */

typedef struct raster_job {
    const void* d_points; /* device (n, 2) array, borrowed until the call returns */
    int64_t n;
    raster_dtype dt;
    int32_t precision; /* used when scale <= 0 */
    double scale;      /* > 0: use this scale instead of 10^precision */
    uint32_t tau, mu;
} raster_job;

/* Cluster many independent point sets together: one fused contraction over
 * all jobs' points, then segmented threshold / agglomeration / filter passes,
 * replayed from a captured HIP graph when the batch fits the captured shape.
 * outs[i] receives job i's result, identical to raster_cluster on that job
 * alone.  On failure every outs[i] is NULL. */
raster_status raster_cluster_batch(const raster_job* jobs, int32_t n_jobs, hipStream_t stream,
                                   raster_result** outs);
/* Same, with options per job: opts[i] (n_jobs entries, or NULL for the
 * defaults everywhere) gives job i's metric, delta and square_step, and
 * outs[i] is identical to raster_cluster_opts on that job alone.  Jobs that
 * share their options run as one fused batch; the groups run one after
 * another, in order of first appearance.  E_INVAL for invalid options and for
 * dims = 3 (batches take two-dimensional points). */
raster_status raster_cluster_batch_opts(const raster_job* jobs, const raster_options* opts, int32_t n_jobs,
                                        hipStream_t stream, raster_result** outs);

/* ---- served form ------------------------------------------------------------- */

/* A serving loop on its own host thread: jobs are admitted while their device
 * memory fits budget_bytes, grouped into batches as they arrive, and run on up
 * to max_slots HIP streams at once, so that new jobs overlap jobs already on
 * the GPU.  Tables stay resident and are reused across jobs. */
raster_status raster_server_create(size_t budget_bytes, int32_t max_slots, raster_server** srv);
/* Queue a job whose points were produced by work on `stream` (0: the null
 * stream).  Submission records an event on `stream` and returns at once; the
 * job's device work waits for that event, so points written by kernels or
 * copies enqueued on `stream` before the call are read only once they are
 * complete.  Its points are borrowed until raster_server_wait returns it.
 * At submission the server enqueues a distinct-tile sketch of the points (one
 * read of them, on its own stream); when the job reaches the head of the
 * queue, its device footprint is computed from that estimate -- the table
 * sized from it with room for one growth step, the binning and spill scratch
 * of its points, the compact arrays and the rows -- and the job is admitted
 * once the running batches, the buffers the idle engines keep and the job
 * fit the budget (an idle engine gives its buffers back to make room).  So the
 * library's in-use device memory stays within budget_bytes while the server
 * runs (raster_memory_stats).  Returns RASTER_E_BUDGET when even the smallest
 * footprint of the job (one distinct tile) exceeds the budget; a job whose
 * estimated footprint exceeds it fails with RASTER_E_BUDGET at
 * raster_server_wait.  E_INVAL for invalid options and for dims = 3. */
raster_status raster_server_submit_stream(raster_server* srv, const raster_job* job, const raster_options* opts,
                                          hipStream_t stream, uint64_t* ticket);
/* raster_server_submit_stream on the null stream with the default options. */
raster_status raster_server_submit(raster_server* srv, const raster_job* job, uint64_t* ticket);
/* Same, with the job's options (metric, delta, square_step; NULL: the
 * defaults), on the null stream: its result is identical to
 * raster_cluster_opts on the job alone.  Jobs that share a batch are grouped
 * by options as in raster_cluster_batch_opts. */
raster_status raster_server_submit_opts(raster_server* srv, const raster_job* job, const raster_options* opts,
                                        uint64_t* ticket);
/* Block until the job behind ticket is done; *latency_s receives submit-to-
 * completion wall time.  Each ticket may be waited on once. */
raster_status raster_server_wait(raster_server* srv, uint64_t ticket, raster_result** out,
                                 double* latency_s);
/* The server's budget and the largest device footprint it has charged at
 * once (running batches plus the buffers idle engines keep). */
raster_status raster_server_memory(raster_server* srv, size_t* budget, size_t* peak_charged);
/* Drain queued work, stop the loop and release the server's memory. */
void raster_server_destroy(raster_server* srv);

/* ---- misc ------------------------------------------------------------------- */

/* Device memory held by the library on the calling thread's current device:
 * bytes in use (tables, scratch, results not yet freed, buffers the batch
 * engines keep), bytes cached for reuse, and the largest in-use figure since
 * the last reset (reset_peak != 0 starts a new window at the current use). */
raster_status raster_memory_stats(size_t* used, size_t* cached, size_t* peak_used, int32_t reset_peak);
raster_status raster_set_tuning(const raster_tuning* t); /* NULL restores defaults */
raster_status raster_get_tuning(raster_tuning* t);
const char* raster_status_string(raster_status s);
const char* raster_last_error(void); /* thread-local detail of the last failure */
const char* raster_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RASTER_H */
