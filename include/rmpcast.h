/*
 * rmpcast.h -- C ABI of the MI355X raycast-and-policy library (librmpcast.so).
 *
 * The library evaluates the raycasting obstacle-avoidance policy of Pantic et al.,
 * "Obstacle avoidance using raycasting and Riemannian Motion Policies at kHz rates for
 * MAVs": for a robot state (position x, velocity xdot) it casts N Halton rays through a
 * voxel map kept on the GPU, evaluates one obstacle policy (f_i, A_i) per ray, metric-sums
 * them and resolves  f = (sum A_i)^+ sum A_i f_i  (Sec. III-A Eq. 1, Sec. III-E Eq. 11).
 * The LiDAR variant takes beam directions and ranges from a point cloud instead of casting
 * rays (Sec. III-G).  All GPU work runs in the library's own HIP kernels for gfx950.
 *
 * Conventions for every call:
 *   - Every call returns an rmpc_status.  On error nothing is written to any output and
 *     rmpc_last_error() (thread-local) describes the failure.
 *   - "dev" pointers are device memory of the context's GPU; "host" pointers are ordinary
 *     host memory.  The library never frees memory it did not allocate.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Blocking calls enqueue on
 *     it and synchronise it before returning.
 *   - A context is used by one thread at a time.
 *   - Lengths are metres, times seconds, velocities metres per second.
 */
#ifndef RMPCAST_H
#define RMPCAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmpc_ctx rmpc_ctx;

typedef enum {
    RMPC_OK = 0,
    RMPC_E_INVALID = -1,        /* bad argument: NULL, NaN/Inf, size out of range, bad dtype */
    RMPC_E_NOMAP = -2,          /* unknown or released map id */
    RMPC_E_OUT_OF_BOUNDS = -3,  /* query position outside the map's grid */
    RMPC_E_NOMEM = -4,          /* the caller's device arena has no room */
    RMPC_E_HIP = -5,            /* a HIP runtime call failed */
    RMPC_E_STOPPED = -6         /* no serving loop is running, or it stopped after an error */
} rmpc_status;

/* Voxel storage (reading: a voxel is occupied when its TSDF value at the centre is <= 0;
 * for occupancy bytes when the byte is non-zero). */
typedef enum {
    RMPC_TSDF_F32 = 0,          /* float32 truncated signed distance */
    RMPC_TSDF_F16 = 1,          /* IEEE binary16 bit patterns (uint16) */
    RMPC_OCC_U8 = 2             /* uint8 occupancy */
} rmpc_dtype;

/* A dense voxel grid.  Voxel (i, j, k) has its centre at origin_m + (idx + 1/2) voxel_m and
 * logical index lin = i + nx * (j + ny * k) (x fastest). */
typedef struct {
    int32_t nx, ny, nz;
    int32_t dtype;              /* rmpc_dtype */
    double voxel_m;
    double origin_m[3];         /* world coordinate of the grid's minimum corner */
} rmpc_map_desc;

/* Policy parameters: the Table I columns ("Static Map" or "LiDAR") plus constants the paper
 * leaves open. */
typedef struct {
    double c;                   /* soft-normalisation parameter (Eq. 4) */
    double eta_rep, nu_rep;     /* repulsive gain and length scale (Eq. 6) */
    double eta_damp, nu_damp;   /* damping gain and length scale (Eq. 8) */
    double radius;              /* policy radius r of the weight w_r (Eq. 9) */
    double eps;                 /* 0 < eps << 1 in the damping denominator (Eq. 8) */
    double max_range_m;         /* rays with no occupied voxel within this range miss */
    double rank_tol;            /* pseudo-inverse keeps eigenvalues > rank_tol * lambda_max */
    double min_range_m;         /* scan points closer than this are skipped */
    int32_t subvoxel;           /* map queries on float32/float16 TSDF maps: non-zero refines
                                   each hit distance to the zero crossing of the trilinearly
                                   interpolated TSDF (the field sampled at eight points from 1.5
                                   voxels before the hit voxel's entry to 2 after it, one secant
                                   step at the first sign change; the paper's raycaster steps a
                                   continuous distance field, Sec. III-E/F); 0: the distance to
                                   the hit voxel's face.  Not allowed on uint8 maps; ignored by
                                   scan queries. */
    int32_t reserved;           /* 0 */
} rmpc_params;

/* Query flags. */
#define RMPC_Q_ILL 1u            /* an eigenvalue within 10x of the pseudo-inverse cut, or the
                                    kept condition number exceeds 1e3 */
#define RMPC_Q_IN_COLLISION 2u   /* the start voxel is occupied: every ray hits at distance 0 */
#define RMPC_Q_TIE 4u            /* some ray carries RMPC_RAY_TIE */

/* Per-ray debug flags (rmpc_trace_debug). */
#define RMPC_RAY_TIE 1u          /* two face crossings within 1e-5 voxel at a decision the
                                    walk took (crossings inside 8^3 cells and 2^3 bricks it
                                    skipped as free are not examined; every decision is exact
                                    regardless) */
#define RMPC_RAY_RANGE_TIE 2u    /* a face crossing within 1e-5 voxel of max_range */
#define RMPC_RAY_START_FACE 4u   /* the start lies within 1e-5 voxel of a face */
#define RMPC_RAY_IN_COLLISION 8u /* the start voxel is occupied */

/* The combined policy of one query (Eq. 1): f = A^+ b with A = sum A_i, b = sum A_i f_i. */
typedef struct {
    double f[3];                /* resolved acceleration, float64 */
    double A[9];                /* sum of per-ray metrics, row major (float32 compensated sums) */
    double b[3];                /* sum of A_i (f_rep,i + f_damp,i) */
    double lambda[3];           /* eigenvalues of A, ascending */
    int32_t rank;               /* eigenvalues kept by the pseudo-inverse */
    int32_t n_hit;              /* rays (or valid scan points) with an obstacle */
    int32_t n_contrib;          /* hits with d < radius and xdot . r > 0 (non-zero metric) */
    int32_t n_tie;              /* rays carrying RMPC_RAY_TIE */
    uint32_t flags;             /* RMPC_Q_* */
    int32_t n_rays;             /* rays cast (or scan points read) */
    int64_t visits;             /* voxels the rays' walks entered, start voxel included (the
                                   walk reads far fewer: it skips free 8^3 cells and 2^3
                                   bricks whole) */
} rmpc_result;

/* Largest ray count per query (the Halton table length). */
#define RMPC_MAX_RAYS 65536

/*
 * rmpc_create -- open a context on GPU `device`.
 *   arena_dev, arena_bytes: a caller-owned device buffer on that GPU from which the library
 *     sub-allocates everything it keeps on the device (maps, the ray-direction table and
 *     the direction-ordered ray lists, about 14 MB together, reduction partials).  It must
 *     stay valid until rmpc_destroy.  At least 16 MiB.
 *   out: receives the context.
 * Computes the float32 Halton direction table (Sec. III-E Eq. 10) for RMPC_MAX_RAYS rays on
 * the device.  Errors: RMPC_E_INVALID (NULL, too small), RMPC_E_HIP.
 */
rmpc_status rmpc_create(int device, void *arena_dev, size_t arena_bytes, rmpc_ctx **out);

/* rmpc_destroy -- release the context's pinned host buffers and the context itself.  The
 * arena stays the caller's.  NULL is accepted. */
rmpc_status rmpc_destroy(rmpc_ctx *ctx);

/*
 * rmpc_map_upload -- make a voxel map resident on the GPU, where every later query reads it
 * (Sec. III-F keeps the map in device memory for all kernels).
 *   desc: grid geometry and storage type; 1 <= nx, ny, nz <= 4096, voxel_m > 0.
 *   voxels: nx*ny*nz elements of the dtype in logical x-fastest order; host memory when
 *     voxels_on_device == 0, device memory of the context's GPU otherwise.  Only read during
 *     the call.
 *   map_id_out: receives an id >= 0.
 * The library keeps the grid as given (x-fastest) in the arena and adds one summary element
 * per whole 8 x 8 x 8 cell and one per whole 2 x 2 x 2 brick (occupied when any of its voxels
 * is), about 1/7 of the grid's size more.  Blocking.
 * Errors: RMPC_E_INVALID, RMPC_E_NOMEM (arena full), RMPC_E_HIP.
 */
rmpc_status rmpc_map_upload(rmpc_ctx *ctx, const rmpc_map_desc *desc, const void *voxels,
                            int voxels_on_device, void *hip_stream, int32_t *map_id_out);

/* rmpc_map_release -- free a map's arena space.  Errors: RMPC_E_NOMAP. */
rmpc_status rmpc_map_release(rmpc_ctx *ctx, int32_t map_id);

/* A sparse map: 8 x 8 x 8-voxel blocks stored only where the world has content (every voxel
 * outside a stored block is free, and the world has no edge), as in the GPU-resident block
 * hash map the paper's system raycasts (Sec. III-E, III-F).  Block (bx, by, bz) covers voxels
 * [8 bx, 8 bx + 8) x [8 by, 8 by + 8) x [8 bz, 8 bz + 8); voxel (i, j, k) has its centre at
 * origin_m + (idx + 1/2) voxel_m, for negative indices too. */
typedef struct {
    int32_t n_blocks;           /* stored blocks, 1 .. 2^22 */
    int32_t dtype;              /* rmpc_dtype of the voxel values */
    double voxel_m;
    double origin_m[3];         /* world position of the minimum corner of voxel (0, 0, 0) */
    double free_value;          /* TSDF maps: the field's value at every voxel outside the stored
                                   blocks (the map's truncation distance, > 0), used by sub-voxel
                                   distances; converted to the storage type as a value would be.
                                   Ignored for uint8 maps. */
} rmpc_sparse_desc;

/*
 * rmpc_sparse_map_upload -- make a sparse map resident on the GPU.
 *   block_coords_host[3 n_blocks]: host int32 (bx, by, bz) of each stored block, each in
 *     [-2^20, 2^20), no block twice.  Block k gets slot k.
 *   values[512 n_blocks]: the voxel values of the dtype, block after block; within block k,
 *     voxel (i, j, l) (0..7 each) at k * 512 + i + 8 j + 64 l.  Host memory when
 *     values_on_device == 0, device memory otherwise.  Only read during the call.
 *   map_id_out: receives the map's id (the same id space as dense maps).
 * The library keeps the values, a 512-bit occupancy mask per block and an open-addressed hash
 * table (a power of two of at least 16 n_blocks entries of 16 bytes, at least 1024) from block
 * coordinates to slots: 16 capacity + 64 n_blocks + 512 elem_bytes n_blocks arena bytes.
 * More than 2^27 blocks: RMPC_E_INVALID.
 * rmpc_query and rmpc_trace_debug accept sparse maps (launch configuration
 * RMPC_CONFIG_SPARSE; the start may lie anywhere whose voxels within max_range keep
 * |index| < 2^23; RMPC_E_OUT_OF_BOUNDS otherwise; sub-voxel distances on TSDF maps read
 * free_value outside the stored blocks); rmpc_trace_debug then reports a hit as
 * slot * 512 + (i + 8 j + 64 l) of the hit voxel in its block.  Batched queries, the serving
 * loop and rollouts (single and batched) take sparse maps too: in a batch a sparse query uses
 * the batch's segmentation with block rounds of 4 steps.  The distance transform takes dense
 * maps only (RMPC_E_INVALID).  Blocking.
 * Errors: RMPC_E_INVALID (NULL, n_blocks, dtype, voxel size, free_value, coordinates, a
 * repeated block), RMPC_E_NOMEM (arena full), RMPC_E_HIP.
 */
rmpc_status rmpc_sparse_map_upload(rmpc_ctx *ctx, const rmpc_sparse_desc *desc, const int32_t *block_coords_host,
                                   const void *values, int values_on_device, void *hip_stream,
                                   int32_t *map_id_out);

/*
 * rmpc_map_footprint -- arena bytes that rmpc_map_upload of this grid takes (the grid plus its
 * cell and brick summaries, before the arena's 256-byte rounding), for sizing an arena.  Makes
 * no GPU call.  The same descriptor checks as rmpc_map_upload apply; in particular the grid
 * must hold fewer than 2^31 voxels (linear indices are int32).
 * Errors: RMPC_E_INVALID.
 */
rmpc_status rmpc_map_footprint(const rmpc_map_desc *desc, size_t *bytes);

/*
 * rmpc_query -- the raycasting policy P_ray of one robot state (Sec. III-E Eq. 11).
 *   x, v: position (world, metres) and velocity, float64 host arrays of 3.
 *   n_rays: 1 <= n_rays <= RMPC_MAX_RAYS; rays are Halton indices 0 .. n_rays-1.
 *   params: policy parameters (all finite; c, nu_rep, nu_damp, radius, eps, max_range_m > 0).
 *   out: host struct receiving the combined policy.
 * The start grid coordinate is g = float32((x - origin) / voxel_m).  A ray's distance is
 * where it enters the first occupied voxel (3-D DDA); rays with none within max_range_m or
 * leaving the grid contribute nothing.  Blocking.
 * Errors: RMPC_E_INVALID, RMPC_E_NOMAP, RMPC_E_OUT_OF_BOUNDS, RMPC_E_HIP.
 */
rmpc_status rmpc_query(rmpc_ctx *ctx, int32_t map_id, const double x[3], const double v[3],
                       int32_t n_rays, const rmpc_params *params, void *hip_stream,
                       rmpc_result *out);

/*
 * rmpc_scan_query -- the LiDAR policy (Sec. III-G): each point p gives direction p/|p| and
 * distance |p|.
 *   points_dev: n_points x 3 float32 on the device, robot-relative in a world-aligned frame;
 *     non-finite points and points with |p| < min_range_m (dropouts as (0,0,0)) are skipped.
 *   n_points: 0 <= n_points <= 2^24.
 *   v: velocity in the same frame.  Blocking.
 * Errors: RMPC_E_INVALID, RMPC_E_HIP.
 */
rmpc_status rmpc_scan_query(rmpc_ctx *ctx, const float *points_dev, int32_t n_points,
                            const double v[3], const rmpc_params *params, void *hip_stream,
                            rmpc_result *out);

/*
 * rmpc_scan_query_noalloc -- rmpc_scan_query for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving or control loops, harnesses that forbid allocation):
 * needs no context and allocates nothing.  Its reduction scratch (block partials of at most
 * 128 blocks and an arrival ticket, 16,640 bytes) is a fixed device array of the library that
 * each GPU holds until the process ends; the call clears what must start at zero.
 *   device: the GPU that holds points_dev and out_dev.
 *   points_dev, n_points, v, params: as for rmpc_scan_query (0 <= n_points <= 2^24).
 *   out_dev: device memory receiving the result, written in stream order: it is complete once
 *     hip_stream reaches the end of this call's work.  The call returns after enqueueing (it
 *     does not wait).
 * The result equals rmpc_scan_query's bit for bit.  Calls that overlap on one GPU (other
 * streams, or other host threads, without ordering between them) share the scratch and race:
 * order them on one stream.
 * Errors: RMPC_E_INVALID (NULL, size out of range, bad parameter), RMPC_E_HIP.
 */
rmpc_status rmpc_scan_query_noalloc(int device, const float *points_dev, int32_t n_points,
                                    const double v[3], const rmpc_params *params, void *hip_stream,
                                    rmpc_result *out_dev);

/*
 * rmpc_trace_debug -- per-ray traversal results of a query, for parity tests.
 *   hit_lin_dev[n_rays]: logical index of the hit voxel, -1 on a miss.
 *   dist_dev[n_rays]: distance in metres to where the ray enters it (float64), +inf on a miss.
 *   flags_dev[n_rays]: RMPC_RAY_* flags.
 *   visits_dev[n_rays]: voxels the ray's walk entered (start voxel included); may be NULL.
 * All output buffers are device memory.  Only params->max_range_m and params->subvoxel (then
 * dist_dev holds the refined distances) are used.  Blocking.
 * Errors: as rmpc_query.
 */
rmpc_status rmpc_trace_debug(rmpc_ctx *ctx, int32_t map_id, const double x[3], int32_t n_rays,
                             const rmpc_params *params, void *hip_stream, int32_t *hit_lin_dev,
                             double *dist_dev, uint8_t *flags_dev, int32_t *visits_dev);

/* A query of a batch. */
#define RMPC_KIND_MAP 0
#define RMPC_KIND_SCAN 1
typedef struct {
    int32_t kind;               /* RMPC_KIND_MAP or RMPC_KIND_SCAN */
    int32_t map_id;             /* map queries: the resident map */
    int32_t n;                  /* map queries: rays (1..65536); scan queries: points (0..2^24) */
    int32_t reserved;
    double x[3];                /* map queries: position (world, metres) */
    double v[3];                /* velocity */
    const float *points_dev;    /* scan queries: n x 3 float32 on the device (robot-relative) */
} rmpc_query_desc;

/* Launch configuration (rmpc_config_set, rmpc_tune_batch).  Hits, distances, visits and the
 * metric sums do not depend on lookahead, blocks_per_cu or use_graph; the segmentation
 * (lane_target_log2) changes only the summation order.  RMPC_RAY_TIE / n_tie may change with
 * the lookahead and the segmentation (they report near-ties at the decisions the walk takes). */
#define RMPC_CONFIG_QUERY 0     /* rmpc_query and rmpc_trace_debug */
#define RMPC_CONFIG_BATCH 1     /* rmpc_query_batch */
#define RMPC_CONFIG_SPARSE 2    /* rmpc_query and rmpc_trace_debug on sparse maps (blocks_per_cu and
                                   use_graph unused) */
typedef struct {
    int32_t lookahead;          /* steps (voxels, free bricks or free cells) planned per
                                   round: 4, 8 or 16 */
    int32_t lane_target_log2;   /* split rays into segments until a query has ~2^this lanes (10..22) */
    int32_t blocks_per_cu;      /* batches: resident blocks per CU of the persistent kernel (0 = max) */
    int32_t use_graph;          /* batches: 1 = replay the launch from a captured hipGraph */
} rmpc_launch_config;

/*
 * rmpc_query_batch -- many map and scan queries in one persistent fused launch (the
 * combination of Sec. III-E/III-G applied to each query independently).
 *   q[n]: queries, 1 <= n; map queries use map_params, scan queries scan_params (either may
 *     be NULL if no query of that kind is present).
 *   out[n]: host results, the same as rmpc_query / rmpc_scan_query would return for each
 *     query alone; bitwise identical when the launch configuration is the same (for a query
 *     on a sparse map: RMPC_CONFIG_SPARSE with lookahead 4 and the batch's lane target).
 * Queries are validated first; any invalid one fails the whole call (the message names its
 * index) and nothing is written.  Large batches are split into several launches.  Blocking.
 * Errors: RMPC_E_INVALID, RMPC_E_NOMAP, RMPC_E_OUT_OF_BOUNDS, RMPC_E_NOMEM, RMPC_E_HIP.
 */
rmpc_status rmpc_query_batch(rmpc_ctx *ctx, const rmpc_query_desc *q, int32_t n,
                             const rmpc_params *map_params, const rmpc_params *scan_params,
                             void *hip_stream, rmpc_result *out);

/* rmpc_config_set / _get -- the launch configuration of single queries on dense maps (which =
 * RMPC_CONFIG_QUERY), of batches (RMPC_CONFIG_BATCH) or of single queries on sparse maps
 * (RMPC_CONFIG_SPARSE).  Errors: RMPC_E_INVALID. */
rmpc_status rmpc_config_set(rmpc_ctx *ctx, int32_t which, const rmpc_launch_config *cfg);
rmpc_status rmpc_config_get(rmpc_ctx *ctx, int32_t which, rmpc_launch_config *cfg);

/*
 * rmpc_tune_batch -- time rmpc_query_batch on this batch for a grid of configurations
 * (lookahead, segmentation target, resident blocks) and keep the fastest as the context's
 * RMPC_CONFIG_BATCH (use_graph is kept as set).
 *   cache_path: optional JSON file; a configuration cached there under this GPU's
 *     architecture, the batch's storage types and its mean ray count bucket is used without
 *     timing, and a newly timed one is added.  NULL: no file.
 *   best: optional, receives the chosen configuration.
 * Runs the batch several times.  Errors: as rmpc_query_batch.
 */
rmpc_status rmpc_tune_batch(rmpc_ctx *ctx, const rmpc_query_desc *q, int32_t n,
                            const rmpc_params *map_params, const rmpc_params *scan_params,
                            void *hip_stream, const char *cache_path, rmpc_launch_config *best);

/* rmpc_directions -- copy the first n (1 <= n <= RMPC_MAX_RAYS) ray directions, float32
 * x,y,z triples, into host memory out_host[3n] (Sec. III-E Eq. 10). */
rmpc_status rmpc_directions(rmpc_ctx *ctx, int32_t n, float *out_host);

/*
 * rmpc_set_profiling -- measurement aid.  While enabled, each rmpc_query / rmpc_scan_query
 * kernel is launched with a start and a stop event recorded by its own dispatch, and its
 * duration is added to a running total.  Enabling (or disabling) resets the total.
 * Errors: RMPC_E_INVALID, RMPC_E_HIP.
 */
rmpc_status rmpc_set_profiling(rmpc_ctx *ctx, int enable);

/* rmpc_get_profile -- total kernel time in milliseconds and number of timed launches since
 * profiling was last enabled.  Errors: RMPC_E_INVALID. */
rmpc_status rmpc_get_profile(rmpc_ctx *ctx, double *kernel_ms, int64_t *launches);

/*
 * Serving loop.  A library thread owns a pool of launch slots, each with its own stream and
 * batch buffers.  Requests submitted from any thread wait in one FIFO queue; whenever a slot
 * is free, the thread takes requests from the front of the queue (up to the slot's query and
 * tile capacity, and while their scan points fit the staging memory) into one persistent
 * launch (the same kernel as rmpc_query_batch), so launches on different slots overlap on
 * the device and new requests join the next launch while earlier ones run (continuous
 * batching).  Each result is the one rmpc_query_batch gives for the request with the same
 * launch configuration.  While the server runs, maps cannot be uploaded or released.
 */
typedef struct {
    rmpc_query_desc q;          /* the query (rmpc_query_batch's descriptor) */
    const float *points_host;   /* scan queries: q.n x 3 float32 in host memory, copied to the
                                   device by the server (q.points_dev is then ignored); NULL to
                                   use q.points_dev.  Either buffer must stay valid and
                                   unchanged until the request is done, and device points must
                                   be complete when rmpc_submit is called.  Pinned host memory
                                   is copied asynchronously, pageable memory synchronously. */
} rmpc_request;

typedef struct {
    int32_t n_slots;            /* launches in flight at once, each on its own stream: 1..8 */
    int32_t max_batch;          /* requests per launch: 1..4096 */
    int32_t max_tiles;          /* 256-lane tiles per launch (0 = 262144); a request needing
                                   more is refused.  Each slot holds 128 B per tile. */
    int32_t max_pending;        /* queued requests before rmpc_submit refuses (0 = 65536) */
    size_t staging_bytes;       /* device memory for host scan points (0 = none) */
    rmpc_params map_params;     /* policy of map requests */
    rmpc_params scan_params;    /* policy of scan requests */
    rmpc_launch_config launch;  /* as for batches */
} rmpc_server_config;

typedef struct {
    uint64_t submitted;         /* requests accepted */
    uint64_t completed;         /* requests with a result (polled or not) */
    uint64_t launches;          /* kernel launches */
    uint64_t pending;           /* requests queued now */
    uint64_t in_flight;         /* requests in running launches now */
    uint64_t refused;           /* submits refused because the queue was full */
    uint64_t staging_waits;     /* launches closed early because staging memory was full */
    uint64_t staging_peak;      /* most staging bytes in use at once */
    uint64_t batch_max;         /* most requests in one launch */
} rmpc_server_counters;

/*
 * rmpc_server_start -- start the serving loop on this context.  Slots, their buffers and the
 * staging memory come from the arena.  Before it returns, every slot's stream makes copies
 * from pinned host memory into the staging memory (queued up to twice the depth of a launch of
 * max_batch scans, at most 1,024) and one empty launch, so that the runtime's one-time set-up
 * of a stream does not delay served requests; this takes milliseconds.  Slot streams stay with
 * the context after rmpc_server_stop and serve the next server.  Errors: RMPC_E_INVALID (bad
 * config, already running), RMPC_E_NOMEM (arena too small), RMPC_E_HIP.
 */
rmpc_status rmpc_server_start(rmpc_ctx *ctx, const rmpc_server_config *cfg);

/*
 * rmpc_submit -- validate a request and queue it; never waits for the device.  Thread-safe.
 *   ticket: receives the request's ticket (increasing in submission order).
 * The latency clock of the request starts here.  Errors: as rmpc_query_batch for an invalid
 * query (nothing is queued), RMPC_E_NOMEM (queue full, or scan points larger than the
 * staging memory), RMPC_E_STOPPED (no server, or it failed; rmpc_last_error says why).
 */
rmpc_status rmpc_submit(rmpc_ctx *ctx, const rmpc_request *req, uint64_t *ticket);

/*
 * rmpc_poll -- non-blocking check of one request.  Thread-safe.
 *   done: 1 if the result is ready (out and latency_s are then written and the ticket is
 *     retired), else 0.
 *   latency_s: optional, seconds from rmpc_submit to the server seeing the result in host
 *     memory.
 * Errors: RMPC_E_INVALID (unknown or retired ticket), RMPC_E_STOPPED.
 */
rmpc_status rmpc_poll(rmpc_ctx *ctx, uint64_t ticket, rmpc_result *out, int32_t *done, double *latency_s);

/*
 * rmpc_poll_completed -- collect up to max ready results in completion order (tickets,
 * out, latency_s: arrays of max entries; latency_s may be NULL) and retire their tickets.
 * Thread-safe.  Errors: RMPC_E_INVALID, RMPC_E_STOPPED.
 */
rmpc_status rmpc_poll_completed(rmpc_ctx *ctx, int32_t max, uint64_t *tickets, rmpc_result *out,
                                double *latency_s, int32_t *n_out);

/* rmpc_server_stats -- the server's counters.  Thread-safe.  Errors: RMPC_E_STOPPED. */
rmpc_status rmpc_server_stats(rmpc_ctx *ctx, rmpc_server_counters *out);

/*
 * rmpc_server_stop -- finish every queued and running request, then stop the thread and
 * return the slots and staging memory to the arena.  Results not yet polled are discarded.
 * Errors: RMPC_E_STOPPED (not running); a failure of the loop is reported as RMPC_E_HIP.
 */
rmpc_status rmpc_server_stop(rmpc_ctx *ctx);

/* ------------------------------------------------------------------------------------------
 * Closed-loop rollout: the ray policy summed with the goal attractor of Sec. III-C (Eq. 3,
 * metric I; s of Eq. 4 with params->c), resolved (Eq. 1) and integrated step by step, as the
 * paper's simulated flights do (Sec. IV-A).
 * ------------------------------------------------------------------------------------------ */

typedef struct {
    double goal[3];             /* goal position, world metres */
    double alpha, beta;         /* attractor gain and damping (> 0) */
    double dt;                  /* integration step, s (> 0) */
    int32_t max_steps;          /* >= 0 */
    double goal_tol;            /* success radius around the goal, m (>= 0) */
    double ray_weight;          /* >= 0: multiplies the ray sums A, b before the attractor is
                                   added (1: Eq. 1 as written; N_ref / n_rays weighs the ray
                                   policy as if N_ref rays were cast) */
    int32_t smooth_every;       /* >= 1: the smoothness is measured on the states every
                                   smooth_every steps (1: every integration step) */
} rmpc_rollout_params;

#define RMPC_ROLLOUT_GOAL 1u       /* the state came within goal_tol of the goal */
#define RMPC_ROLLOUT_COLLISION 2u  /* the state's voxel is occupied */
#define RMPC_ROLLOUT_LEFT_GRID 3u  /* the state left the grid */
#define RMPC_ROLLOUT_TIMEOUT 4u    /* max_steps steps taken */

typedef struct {
    uint32_t status;            /* RMPC_ROLLOUT_* */
    int32_t n_steps;            /* integration steps taken */
    double smoothness;          /* mean of 1 - angle / pi between consecutive non-zero
                                   displacements of the sampled states x_0, x_m, x_2m, ...
                                   (m = smooth_every; 1 with fewer than two such displacements;
                                   Sec. IV-B's path smoothness) */
    double path_length_m;
    double x[3], v[3];          /* final state */
} rmpc_rollout_result;

/*
 * rmpc_rollout -- fly from (x0, v0) toward rp->goal.  Each step k: stop when within goal_tol of
 * the goal (RMPC_ROLLOUT_GOAL) or outside the grid (RMPC_ROLLOUT_LEFT_GRID); run the query of
 * (x_k, v_k) with n_rays rays (rmpc_query) and stop when its voxel is occupied
 * (RMPC_ROLLOUT_COLLISION); then a_k = (I + w A)^-1 (f_a + w b) in float64, with A, b the
 * query's sums, w = ray_weight and f_a = alpha s(goal - x_k) - beta v_k, and v_{k+1} = v_k + a_k dt,
 * x_{k+1} = x_k + v_{k+1} dt.  After max_steps steps the status is RMPC_ROLLOUT_TIMEOUT (or GOAL
 * if the last state is within goal_tol).
 *   traj_host: NULL, or a host array of (max_steps + 1) x 6 doubles receiving x, v of every state
 *     (row k = state k; rows past out->n_steps are left untouched).
 *   out: the outcome.  Blocking (one query per step).
 * Errors: those of rmpc_query other than RMPC_E_OUT_OF_BOUNDS; RMPC_E_INVALID for bad rp.
 */
rmpc_status rmpc_rollout(rmpc_ctx *ctx, int32_t map_id, const double x0[3], const double v0[3], int32_t n_rays,
                         const rmpc_params *params, const rmpc_rollout_params *rp, void *hip_stream,
                         double *traj_host, rmpc_rollout_result *out);

/*
 * rmpc_edt -- the exact Euclidean distance transform of a resident map's occupancy: the
 * distance field that the ESDF single-lookup policy of Sec. III-D reads.
 *   sqdist_dev[nx * ny * nz]: device memory (x fastest, as the map), receives for every voxel
 *     the squared distance, in voxels, from its centre to the centre of the nearest occupied
 *     voxel (an integer; 0 on occupied voxels), or -1 everywhere when no voxel is occupied.
 * Dense maps only.
 * Runs on hip_stream and waits for it.  Errors: RMPC_E_INVALID, RMPC_E_NOMAP, RMPC_E_HIP.
 */
rmpc_status rmpc_edt(rmpc_ctx *ctx, int32_t map_id, int32_t *sqdist_dev, void *hip_stream);

/*
 * rmpc_esdf_query -- the single-lookup ESDF policy of Sec. III-D (the paper's baseline): at
 * x, the distance d of x's voxel read from sqdist_dev (rmpc_edt of this map: d = h sqrt(q)),
 * the gradient by central differences over the six neighbour voxels (indices clamped at the
 * grid edge, divided by 2h), the obstacle direction r = -grad / |grad|, and one obstacle
 * policy (Eqs. 4-9, params as for map queries) for (r, d), resolved as a query is.  out: the
 * result (A, b, f, lambda, rank; n_hit = 1 when a policy was evaluated, n_contrib as for a
 * ray; n_rays = 1; RMPC_Q_IN_COLLISION when x's voxel is occupied).  A grid with nothing
 * occupied, or a zero gradient, gives zero sums.  float64 on the device.  Blocking.
 * Errors: RMPC_E_INVALID, RMPC_E_NOMAP, RMPC_E_OUT_OF_BOUNDS, RMPC_E_HIP.
 */
rmpc_status rmpc_esdf_query(rmpc_ctx *ctx, int32_t map_id, const int32_t *sqdist_dev, const double x[3],
                            const double v[3], const rmpc_params *params, void *hip_stream, rmpc_result *out);

/* A flight of a batched rollout. */
typedef struct {
    int32_t map_id;
    int32_t n_rays;             /* rays per query, 1..65536 */
    double x0[3], v0[3];        /* start state */
    rmpc_rollout_params rp;     /* goal, gains, step, limits of this flight */
} rmpc_flight;

/*
 * rmpc_rollout_batch -- n independent flights (each as rmpc_rollout defines it) advanced
 * together: every step runs the queries of all flights still flying as one rmpc_query_batch
 * launch, so n flights cost about as many launches as the longest one has steps.
 *   flights[n], out[n]: host arrays, 1 <= n.  A flight leaves the batch when it ends; the
 *   others are unaffected.
 * Each flight's outcome is bit for bit the one rmpc_rollout gives when the batch launch
 * configuration (RMPC_CONFIG_BATCH) equals the query configuration (RMPC_CONFIG_QUERY).
 * Every flight is validated first (unknown map, n_rays, parameters); any invalid one fails the
 * call with its index in the message and nothing is written.  Blocking.
 * Errors: RMPC_E_INVALID, RMPC_E_NOMAP, and those of rmpc_query_batch.
 */
rmpc_status rmpc_rollout_batch(rmpc_ctx *ctx, const rmpc_flight *flights, int32_t n, const rmpc_params *params,
                               void *hip_stream, rmpc_rollout_result *out);

/* rmpc_last_error -- text of the calling thread's last error ("" if none). */
const char *rmpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RMPCAST_H */
