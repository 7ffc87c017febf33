/*
 * flic.h -- FLIC range-image clustering on AMD Instinct MI355X (gfx950).
 *
 * FLIC (Hasecke, Hahn, Kummert, "FLIC: Fast Lidar Image Clustering", arXiv
 * 2003.00575) segments a Lidar range image into object instances:
 *
 *   1. Edge test (Section III.B, Eq. 3/4).  Two pixels are connected when
 *        D^2 = (d1*d1 + d2*d2) - ((2*cos a) * (d1*d2)) <= T^2
 *      in IEEE binary32, each operation rounded to nearest-even, no fused
 *      multiply-add, T^2 = fl32(T*T), ordered compare (NaN never connects).
 *      Neighbours are the same column k rows below and the same row k columns
 *      to the right with 360-degree wrap, for k = 1..N: k = 1 is the direct
 *      4-neighbourhood (Section III.B.1), k >= 2 the map / skip connections
 *      of Section III.B.2 applied to every pixel.
 *   2. Pixels whose range is not (> 0 and finite) are missing measurements
 *      (Section III.A, zero = removed) and take part in no edge.
 *   3. Connected-component labelling over those edges (Section III.B.1), with
 *      canonical labels: every measurement gets the smallest linear index
 *      r*W + c of its component; missing pixels get -1.  The result is unique,
 *      so every entry point returns the same bits for the same input.
 *   4. Optional cluster-size threshold (Section III.B.1, 100 points in the
 *      paper): with min_points > 0, every pixel of a component with fewer
 *      than min_points measurements gets -1 as well.
 *
 * Conventions for every entry point:
 *   - Device pointers are HIP device addresses on the context's device.
 *     The caller owns every buffer; the library never frees or keeps a
 *     caller pointer beyond completion of the work it enqueued.
 *   - range and labels_out must not overlap each other or the tables.
 *   - Arguments are validated on the host before any HIP call; an invalid
 *     argument returns FLIC_EINVAL and leaves labels_out untouched.
 *   - Failed HIP runtime calls return FLIC_EHIP; flic_last_error() then gives
 *     a message (thread-local, valid until the next call on the thread).
 *   - A context is used by one host thread at a time.
 */
#ifndef FLIC_H
#define FLIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t flic_status;
#define FLIC_OK 0
#define FLIC_EINVAL (-1)  /* invalid argument, nothing enqueued              */
#define FLIC_ENOMEM (-2)  /* allocation failed or HBM budget exceeded         */
#define FLIC_EHIP (-3)    /* HIP runtime error, see flic_last_error()         */

#define FLIC_MAX_SKIP 8

/* Angle tables supplied by the caller (the sensor's channel and azimuth
 * geometry, Section III.B: "provided by the manufacturer").  Device pointers.
 *   cos_v: [N][H] float32; cos_v[(k-1)*H + r] = cos(angle between rows r and
 *          r+k); entries with r >= H-k are never read.
 *   cos_h: [N][W] float32; cos_h[(k-1)*W + c] = cos(angle between columns c
 *          and (c+k) mod W).
 * The values are used exactly as given (never recomputed).                  */
typedef struct {
    const float* cos_v;
    const float* cos_h;
} flic_alpha_tables;

/* One scan of a batch.  All pointers are device pointers.
 *   range_img  [H][W] float32 metres, row-major (row = channel, col = azimuth)
 *   H >= 1, W > 2*skip_depth, H*W <= INT32_MAX
 *   threshold  metres, finite, >= 0      skip_depth  N, 1..FLIC_MAX_SKIP
 *   labels_out [H][W] int32, scan-local linear indices
 *   min_points cluster-size threshold of Section III.B.1: 0 = none; > 0 =
 *              components with fewer measurements are labelled -1 (1 keeps
 *              every component but still runs the counting kernels);
 *              < 0 is FLIC_EINVAL.  The library then also keeps an
 *              [H][W] int32 count array in its scratch.
 *   map_connections  0: skip edges from every pixel (offsets 2..N along
 *              both axes); 1: the paper's Map Connections (Section
 *              III.B.2): for each stride k = 2..N, only pixels whose row
 *              and column are multiples of k connect to their k-th
 *              neighbour to the right (with wrap) and below.  Other values
 *              are FLIC_EINVAL.  With skip_depth 1 both are the same.      */
typedef struct {
    const float* range_img;
    int32_t H;
    int32_t W;
    flic_alpha_tables tables;
    float threshold;
    int32_t skip_depth;
    int32_t* labels_out;
    int32_t min_points;
    int32_t map_connections;
} flic_scan;

typedef struct flic_ctx flic_ctx;
typedef struct flic_plan flic_plan;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context itself allocates (descriptor tables, plans); 0 means no
 * cap.  Returns FLIC_EINVAL for a null out-pointer or bad device.           */
flic_status flic_ctx_create(flic_ctx** out, int device, size_t hbm_budget_bytes);

/* Destroy a context after synchronising the device work it enqueued. Plans
 * created from it must be destroyed first.  Null is a no-op.               */
void flic_ctx_destroy(flic_ctx* ctx);

/* Cluster one scan (all pointers device pointers, see flic_scan for the
 * layout) and block until the labels are written.  Uses one default context
 * per HIP device, shared by all host threads (their launches are serialised,
 * their waits are not), on the current device and the null stream.  The single-scan
 * entry points use dense skip edges and no size threshold (map_connections
 * = 0, min_points = 0); flic_cluster_batched with n = 1 takes the others.  */
flic_status flic_cluster(const float* range_img, int32_t H, int32_t W,
                         const flic_alpha_tables* alpha_tables,
                         float threshold, int32_t skip_depth,
                         int32_t* labels_out);

/* Stream-ordered form of flic_cluster: enqueues the work on `hip_stream`
 * (a hipStream_t, or null for the null stream) and returns at once.  The
 * table pointers are read on the host during the call; the device buffers
 * must stay valid until the stream reaches the end of the work.             */
flic_status flic_cluster_async(flic_ctx* ctx, const float* range_img,
                               int32_t H, int32_t W,
                               const flic_alpha_tables* alpha_tables,
                               float threshold, int32_t skip_depth,
                               int32_t* labels_out, void* hip_stream);

/* Allocation-free form of flic_cluster_async, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): no context, and no allocation of
 * any kind.  Its scratch is a fixed device array of 16 MiB per device
 * (FLIC_NOALLOC_SCRATCH_BYTES), reserved by the library until the process
 * ends; a scan whose scratch exceeds it (tile pass masks and run roots,
 * border slots and a 4-byte-per-pixel parent array: a 128 x 4096 scan at
 * skip depth 8 needs about 3.4 MiB) returns FLIC_EINVAL with nothing
 * enqueued.  Enqueues on `hip_stream` (null: the null stream) on the current
 * device and returns at once.  All calls on one device share that array, so
 * calls whose work overlaps on the device race and give wrong labels: order
 * them on one stream, or wait for one before starting the next.  Same
 * arguments, validation and labels as flic_cluster_async.                   */
#define FLIC_NOALLOC_SCRATCH_BYTES (16u << 20)
flic_status flic_cluster_noalloc(const float* range_img, int32_t H, int32_t W,
                                 const flic_alpha_tables* alpha_tables,
                                 float threshold, int32_t skip_depth,
                                 int32_t* labels_out, void* hip_stream);

/* Cluster n independent scans of any shapes, thresholds and skip depths in
 * one stream-ordered sequence of launches (no per-scan launches).  `scans`
 * is a host array read during the call.  Each scan's labels are identical to
 * what flic_cluster returns for it alone.  n == 0 is a no-op.               */
flic_status flic_cluster_batched(flic_ctx* ctx, const flic_scan* scans,
                                 int32_t n, void* hip_stream);

/* flic_cluster_batched for callers whose data lives in host memory: on
 * `hip_stream`, each scan's range image is first copied from
 * host_ranges[i] (H*W float32, row-major) into scans[i].range_img, then the
 * batch is clustered, then each scan's labels are copied to host_labels[i]
 * (H*W int32).  host_ranges or host_labels may be null (no copies that way),
 * and so may single entries.  Host buffers should be pinned (hipHostMalloc)
 * for the copies to be asynchronous; they must stay valid, and untouched,
 * until the stream reaches the last copy.  This is the continuous-batching
 * serving path: one call per batch instead of two copies per frame.
 * Returns like flic_cluster_batched; on an error in a copy, earlier copies
 * and launches may already be enqueued.  Section III.B (the same labels).   */
flic_status flic_cluster_batched_host(flic_ctx* ctx, const flic_scan* scans, int32_t n,
                                      const float* const* host_ranges, int32_t* const* host_labels,
                                      void* hip_stream);

/* Build a reusable plan for batches shaped like `scans` (same n, and per
 * entry the same H, W, skip_depth and min_points > 0 or not): descriptors are laid out once on the
 * device, tile shapes come from the autotune table, and the launch sequence
 * is captured in a hipGraph.                                               */
flic_status flic_plan_create(flic_ctx* ctx, const flic_scan* scans, int32_t n,
                             flic_plan** out);

/* Launch a plan on `hip_stream` for `scans`, which must match the plan's
 * shapes entry by entry: the same H, W, skip_depth and map_connections,
 * and min_points zero where the plan's is zero, positive where it is
 * positive.  Pointers,
 * thresholds and positive min_points values may differ: changed
 * descriptors are uploaded before the graph launch.  FLIC_EINVAL on a
 * shape mismatch.  A plan owns one scratch buffer, so its launches run one
 * after the other: a launch on a different stream from the previous one
 * first waits (on the device, without blocking the host) for that launch.  */
flic_status flic_plan_launch(flic_plan* plan, const flic_scan* scans, int32_t n,
                             void* hip_stream);

/* Destroy a plan (synchronises its last launch).  Null is a no-op.         */
void flic_plan_destroy(flic_plan* plan);

/* Force the tile width (columns per workgroup tile; the tile then holds
 * 8192 / tile_w rows) for every later launch on this context: tile_w is 64,
 * 128 or 256, or 0 to restore the built-in choice by scan shape.  Labels
 * do not depend on it.  Plans keep the width they were created with.       */
flic_status flic_set_tile_override(flic_ctx* ctx, int32_t tile_w);

/* Tile width for scans of exactly this shape and skip depth (an autotuner
 * result): 64, 128 or 256 columns per tile, or 0 to remove the rule.  Rules
 * apply to launches and plans created afterwards on this context; the
 * global override of flic_set_tile_override takes precedence.  Labels do
 * not depend on the tile width.                                            */
flic_status flic_ctx_set_tile_rule(flic_ctx* ctx, int32_t H, int32_t W, int32_t skip_depth,
                                   int32_t tile_w);

/* Plans created afterwards on this context split every group of scans that
 * share a launch configuration (tile width, skip depth, size threshold or
 * not, skip-edge mode) into up to `parts` launch sequences over consecutive
 * scans.  Every sequence is its own branch of the plan's graph (different
 * groups are always separate branches), so that the branches' passes can
 * overlap.  parts 1..64 (1, the default, keeps one sequence per group; on
 * full-GPU batches more parts only add launches); labels do not depend on
 * it.  FLIC_EINVAL otherwise.                                              */
flic_status flic_ctx_set_plan_parts(flic_ctx* ctx, int32_t parts);

/* The tile width the context would use for such a scan.                   */
flic_status flic_ctx_tile_for(const flic_ctx* ctx, int32_t H, int32_t W, int32_t skip_depth,
                              int32_t* tile_w);

/* Descriptor and scratch bytes a flic_cluster_batched call on `scans` would
 * need (only the shapes, skip depths and tile rules matter; pointers are
 * checked like a launch's but never dereferenced).                        */
flic_status flic_batch_bytes(const flic_ctx* ctx, const flic_scan* scans, int32_t n,
                             size_t* desc_bytes, size_t* scratch_bytes);

/* Grow every launch slot of the context to at least these sizes now (within
 * its HBM budget), so later launches never allocate or free device memory.
 * Waits for the slots' previous launches.                                   */
flic_status flic_ctx_reserve(flic_ctx* ctx, size_t desc_bytes, size_t scratch_bytes);

/* Device bytes the context and its plans currently hold (descriptor and
 * scratch buffers); the budget given to flic_ctx_create caps this value.   */
flic_status flic_ctx_bytes_in_use(const flic_ctx* ctx, size_t* bytes);

/* Per-pass timing for measurement.  While enabled, every launch enqueued by
 * flic_cluster_async / flic_cluster_batched on this context records HIP
 * events on its stream around each of its kernels (plans are not timed).
 * flic_ctx_pass_times waits for those events, writes the summed durations
 * in milliseconds of the three passes (tile labelling, border merge,
 * relabel) to total_ms[0..2], the number of timed launches to *n_launches,
 * and starts a new accumulation.                                           */
flic_status flic_ctx_set_pass_timing(flic_ctx* ctx, int32_t enable);
flic_status flic_ctx_pass_times(flic_ctx* ctx, float* total_ms, int32_t* n_launches);

/* Ground extraction (Section III.A), the step before clustering.  Sensor
 * tables (device pointers, H float32 entries each; entry 0 of the first four
 * is never read):
 *   sin_a, cos_a   sin / cos of the angle between rows r-1 and r
 *   tan_lo, tan_hi window of tan(beta) in which the pair (r-1, r) spans a
 *                  near-horizontal surface: the tangents of the upper beam's
 *                  angle below the horizontal minus / plus the threshold angle
 *                  (10 degrees in the paper), the lower end clamped at 0
 *   sin_d, cos_d   sin / cos of row r's elevation angle
 *   sensor_height  metres of the sensor above the wheel plane
 *   tan_theta      slope of the height line (tan 10 degrees in the paper)   */
typedef struct {
    const float* sin_a;
    const float* cos_a;
    const float* tan_lo;
    const float* tan_hi;
    const float* sin_d;
    const float* cos_d;
    float sensor_height;
    float tan_theta;
} flic_ground_tables;

/* Remove the ground from n_scans range images of one shape taken with one
 * sensor (stream-ordered on hip_stream, returns at once).  range_in and
 * range_out are [n_scans][H][W] float32 device buffers that must not
 * overlap; ground_mask is [n_scans][H][W] uint8 (1 = ground) or null.
 * A measurement (range > 0 and finite) is ground when
 *   - Eq. (2), tan(beta) = (d2 sin a) / (d1 - d2 cos a) in binary32 with an
 *     IEEE division, for the pair it forms with the cell above (d1 above,
 *     d2 below), lies in that row's [tan_lo, tan_hi]; a cell in the first
 *     row or under a missing cell takes the pair it forms with the cell below;
 *   - and it lies below the height line: sensor_height + d sin_d[r] <=
 *     (d cos_d[r]) tan_theta.
 * Ground cells get range 0 (removed, as Section III.A treats zeros); every
 * other value is copied unchanged.  The output feeds the flic_cluster*
 * entry points.  H, W >= 1, H*W <= INT32_MAX, n_scans 0..65535 (0 is a
 * no-op; the range pointers may then be null), sensor_height and tan_theta
 * finite, no overlap between inputs and outputs; FLIC_EINVAL otherwise,
 * with nothing enqueued.                                                  */
flic_status flic_ground_remove(flic_ctx* ctx, const float* range_in, int32_t n_scans,
                               int32_t H, int32_t W, const flic_ground_tables* tables,
                               float* range_out, uint8_t* ground_mask, void* hip_stream);

/* ---- Serving runtime --------------------------------------------------------
 * Frames of many sensors clustered continuously on one device, each frame as
 * it arrives (the real-time, scan-by-scan use of Section IV.A), with the
 * frames that are ready at the same time sharing one batched launch.
 *
 * A server owns per sensor its angle tables and slots_per_sensor device frame
 * slots (range and label buffers), admitted against hbm_budget together with
 * the context's launch ring (reserved for max_batch frames of the largest
 * registered shape).  A submitted frame waits FIFO per sensor; beyond
 * max_queue waiting frames the oldest is dropped.  It is admitted when one
 * of its sensor's slots is free.  Whenever one of n_streams launch streams
 * is idle, every admitted frame not yet launched (oldest first, at most
 * max_batch) goes out as one launch on that stream: each frame's range in,
 * one flic_cluster_batched of the frames, each frame's labels back to its
 * host buffer (how the frames move: stage_kernels, below).  Labels are those
 * of flic_cluster (scan-local linear indices, Section III.B, no size
 * threshold, dense skip edges).
 *
 * Times are seconds on the server's clock (flic_server_now: a monotonic clock
 * started at creation).  submit and progress take the current time from the
 * caller, so a driver (or a test) decides when events happen; replay runs a
 * whole arrival schedule in real time.  A server is used by one thread at a
 * time.  Host buffers should be pinned (hipHostMalloc) for the copies to be
 * asynchronous; each must stay valid until its frame is done.  With
 * stage_kernels 1, a batch's frames move between host and device buffers in
 * one kernel launch per direction that reads (writes) the host buffers
 * directly; with 2, the clustering passes themselves read the ranges from
 * and write the labels to the host buffers.  A frame whose buffers the HIP
 * runtime does not report as device-accessible at the same address (or that
 * are not 16-byte aligned) is copied with hipMemcpyAsync instead.  With 2,
 * a frame whose host buffers overlap those of another frame of the same
 * launch goes through its device slot and is copied as with 1.
 *
 * With ctx == NULL the server simulates the device: nothing is allocated or
 * launched, and a launch is done sim_launch_s seconds after it was made
 * (host buffers are then never touched and may be null).                   */
typedef struct flic_server flic_server;

typedef struct {
    int32_t n_streams;        /* launch streams, 1..8                            */
    int32_t max_batch;        /* frames per launch, 1..1024 (1: one launch each) */
    int32_t slots_per_sensor; /* device frame slots per sensor, 1..16            */
    int32_t max_queue;        /* waiting frames per sensor before drops, >= 1    */
    uint64_t hbm_budget;      /* bytes: tables + slots + launch ring; 0 = no cap */
    double sim_launch_s;      /* simulated launch duration (ctx == NULL), >= 0   */
    int32_t stage_kernels;    /* 0: one hipMemcpyAsync per frame and direction;  */
                              /* 1: one copy kernel per batch and direction;     */
                              /* 2: no copies, the passes read and write the     */
                              /* host buffers (see below)                        */
} flic_server_config;

/* One frame's history.  batch is the launch's sequence number (-1 when the
 * frame was dropped or not launched yet); t_done is +inf for a dropped
 * frame and NaN for one not done yet.                                       */
typedef struct {
    int32_t sensor;
    int32_t batch;
    int64_t tag;
    double t_arrival;
    double t_admit;
    double t_launch;
    double t_done;
} flic_frame_record;

/* One scheduled arrival for flic_server_replay: at t seconds after the
 * replay starts, a frame of `sensor` arrives in host_range ([H][W] float32)
 * and its labels go to host_labels ([H][W] int32).                         */
typedef struct {
    double t;
    int32_t sensor;
    int32_t pad_;
    const float* host_range;
    int32_t* host_labels;
} flic_arrival;

/* Create a server on ctx's device (ctx may be NULL: simulated device).  The
 * context stays owned by the caller and must outlive the server.
 * FLIC_EINVAL for a null out-pointer or a config field out of range.       */
flic_status flic_server_create(flic_ctx* ctx, const flic_server_config* cfg, flic_server** out);

/* Register a sensor of H x W frames with skip depth skip_depth and threshold
 * (metres); host_tables holds host pointers to the angle tables in the
 * layout of flic_alpha_tables (copied to the device).  The sensor's id is
 * written to *sensor_out (0, 1, ... in registration order).  FLIC_EINVAL
 * for arguments flic_cluster would reject; FLIC_ENOMEM when the budget or a
 * device allocation does not allow it: nothing of the sensor is kept, but
 * the context's launch ring stays grown if a larger shape made it grow.   */
flic_status flic_server_add_sensor(flic_server* srv, int32_t H, int32_t W, const flic_alpha_tables* host_tables,
                                   float threshold, int32_t skip_depth, int32_t* sensor_out);

/* A frame of `sensor` that arrived at t_arrival; `now` is the current time
 * (its admission time when a slot is free).  tag is returned in its
 * record.  FLIC_EINVAL for an unknown sensor or (with a device) a null
 * buffer.                                                                  */
flic_status flic_server_submit(flic_server* srv, double now, double t_arrival, int32_t sensor,
                               const float* host_range, int32_t* host_labels, int64_t tag);

/* Retire finished launches (their frames are done at `now`, their slots go
 * back to the sensors and waiting frames are admitted), then launch on every
 * idle stream.  *completed (may be null) gets the number of frames retired.
 * FLIC_EHIP on a failed HIP call; the server must then be destroyed.       */
flic_status flic_server_progress(flic_server* srv, double now, int32_t* completed);

/* Run n arrivals (t non-decreasing, relative to the start of the replay) in
 * real time: submit each when its time comes, progress in between, until
 * every frame is done or dropped.  Records keep the arrival times on the
 * server clock.                                                             */
flic_status flic_server_replay(flic_server* srv, const flic_arrival* arrivals, int32_t n);

/* The current time on the server clock.                                    */
double flic_server_now(const flic_server* srv);

/* Records of the frames submitted since creation or the last clear, in
 * submission order: writes min(n_max, count) records to out (out may be
 * null with n_max 0) and the count to *n_out; also the number of dropped
 * frames and of launches (either may be null).                             */
flic_status flic_server_records(const flic_server* srv, flic_frame_record* out, int64_t n_max, int64_t* n_out,
                                int64_t* dropped, int64_t* launches);

/* Forget the records and counters; only while no frame is waiting, admitted
 * or in flight (FLIC_EINVAL otherwise).                                    */
flic_status flic_server_clear(flic_server* srv);

/* Wait for the server's streams, then free everything it allocated.       */
void flic_server_destroy(flic_server* srv);

/* Message for the last error on this thread ("" if none).                  */
const char* flic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
