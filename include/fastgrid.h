/*
 * fastgrid.h — C ABI of libfastgrid.so: FAST corner detection on an image
 * pyramid with 3x3 non-maxima suppression and one feature per grid cell,
 * on an AMD Instinct MI355X (gfx950).
 *
 * The operation follows "Faster than FAST: GPU-Accelerated Frontend for
 * High-Speed VIO" (Nagy, Foehn, Scaramuzza, IROS 2020):
 *   - image pyramid, each level half the previous one (Section II-B, and the
 *     stage list of Section III-C);
 *   - FAST segment test on the 16-pixel radius-3 Bresenham circle with
 *     threshold t (the paper's epsilon) and arc length N (Section II-D, Eq. (1));
 *     corner score 0 when the test fails (Section II-D);
 *   - non-maxima suppression in the 3x3 Moore neighbourhood (Section I-B, n=1);
 *   - one feature per grid cell, the highest score, over all levels on one
 *     shared level-0 grid (Section II-B, Section II-C, Algorithm 1).
 *
 * Exact definitions used where the paper leaves a choice:
 *   - level k+1 pixel = (a+b+c+d+2)>>2 of the 2x2 block of level k; level sizes
 *     are floor halvings (W_k = W_{k-1}/2, H_k = H_{k-1}/2);
 *   - a pixel is tested only if 3 <= x <= W_k-4 and 3 <= y <= H_k-4;
 *   - brighter: p > c + t; darker: p < c - t; corner iff a circular run of at
 *     least N brighter, or of at least N darker, circle pixels exists;
 *   - score = max(sum over brighter circle pixels of (p-c-t),
 *                 sum over darker circle pixels of (c-p-t)), in [N, 4080];
 *   - NMS keeps a pixel iff its score is > 0 and it ranks above all 8
 *     neighbours by (score descending, row-major index ascending);
 *   - the cell of a level-k survivor (x, y) is ((x<<k)/cell, (y<<k)/cell); the
 *     cell keeps its survivor of highest score, then lowest level, then lowest
 *     row-major index at that level.
 *
 * Conventions
 *   - Every call returns int: FAST_OK (0) or a negative FAST_E* code.
 *   - Argument validation is synchronous: on FAST_EINVAL nothing is enqueued.
 *   - Work is enqueued asynchronously on the given stream (a hipStream_t passed
 *     as void*, NULL for the null stream); results are valid after the stream
 *     synchronises or fast_poll reports completion.  Device faults surface as
 *     FAST_EHIP from a later call.
 *   - A submission with a ticket leaves a completion event recorded on its
 *     stream in the context's ring of 256; a later submission that reuses the
 *     entry waits on that event unless fast_poll or fast_wait has already
 *     reported the ticket complete.  Keep such a stream alive until then (the
 *     serving loops' own streams live as long as the context).
 *   - All image planes and output arrays are device memory owned by the
 *     caller; the library never frees them.  The library owns only its context
 *     (job tables, queue counters, events, graphs, scratch).
 *   - One host thread at a time per context.
 */
#ifndef FASTGRID_H
#define FASTGRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FAST_OK = 0,
    FAST_EINVAL = -1,     /* invalid argument; nothing was enqueued */
    FAST_ENOMEM = -2,     /* a library-owned allocation failed */
    FAST_EHIP = -3,       /* a HIP runtime call failed (detail: fast_last_error) */
    FAST_EBUSY = -4,      /* all in-flight slots are taken */
    FAST_ETIMEDOUT = -5   /* fast_wait ran out of time */
};

#define FAST_MAX_LEVELS 8
#define FAST_MAX_CELL 256
#define FAST_MAX_JOBS 4096

typedef struct fast_ctx fast_ctx;          /* opaque, library-owned */

/* One uint8 grayscale plane in device memory: row y starts at data + y*pitch.
 * Requirements: width >= 1, height >= 1, width <= 65535, height <= 65535,
 * pitch >= width, pitch % 16 == 0, (uintptr_t)data % 16 == 0.
 * Bytes between width and pitch are never read as pixels and never written. */
typedef struct {
    uint8_t *data;
    int32_t width;
    int32_t height;
    int32_t pitch;
} fast_plane;

/* One grid-cell result (8 bytes).  x, y are coordinates on pyramid level
 * `level`; the level-0 position is (x << level, y << level).  An empty cell is
 * x = y = 0xFFFF, score = 0, level = 0xFF, reserved = 0. */
typedef struct {
    uint16_t x;
    uint16_t y;
    uint16_t score;
    uint8_t level;
    uint8_t reserved;
} fast_feature;

/* Corner score kinds (Section II-D names three; a pixel that is not a corner
 * by the segment test scores 0 under all of them):
 *   FAST_SCORE_SADB  max(sum over brighter circle points of (p-c-t),
 *                        sum over darker circle points of (c-p-t)), the default;
 *   FAST_SCORE_SADA  the same two sums over only the circle points that lie on
 *                    a continuous arc of at least n points of their label;
 *   FAST_SCORE_MT    the largest d such that n consecutive circle points all
 *                    exceed the centre by at least d, or all fall below it by
 *                    at least d.  The segment test with threshold t' passes
 *                    exactly when d > t', so the maximum passing threshold is
 *                    d - 1; the score is d (t < d <= 255).
 * NMS and the cell arg-max compare scores of the chosen kind. */
#define FAST_SCORE_SADB 0
#define FAST_SCORE_SADA 1
#define FAST_SCORE_MT 2

/* One detection request for the batched entry point. */
typedef struct {
    const fast_plane *pyr;   /* host array of `levels` planes: [0] input, [1..] written */
    int32_t levels;          /* 1..FAST_MAX_LEVELS */
    int32_t t;               /* threshold, 0..255 */
    int32_t n;               /* arc length N, 1..16 */
    int32_t cell;            /* cell side in level-0 pixels, multiple of 2^(levels-1), <= 256 */
    fast_feature *out;       /* device array of gw*gh slots, row-major */
    int32_t score;           /* FAST_SCORE_*; 0 (zero-initialised jobs) is FAST_SCORE_SADB */
} fast_job;

/* Create a context on HIP device `hip_device`.  *out receives the context.
 * Errors: FAST_EINVAL (null out, bad device), FAST_EHIP, FAST_ENOMEM. */
int fast_ctx_create(int hip_device, fast_ctx **out);

/* Destroy a context after its outstanding work has completed (its submissions'
 * events; with a launched live plan, the whole device).  NULL is a no-op. */
void fast_ctx_destroy(fast_ctx *ctx);

/* Static description of a status code. */
const char *fast_strerror(int status);

/* Detail of the last error on this context (e.g. the hipError_t name); the
 * string stays valid until the next call on the context. */
const char *fast_last_error(const fast_ctx *ctx);

/* Level sizes of a pyramid: fills dims[0..levels-1] with data = NULL,
 * width/height the floor halvings, pitch = width rounded up to 64.
 * Errors: FAST_EINVAL (bad sizes, levels out of range, a level of size 0). */
int fast_pyr_dims(int width, int height, int levels, fast_plane *dims);

/* Grid size for a cell: *gw = ceil(width/cell), *gh = ceil(height/cell). */
int fast_grid_dims(int width, int height, int cell, int *gw, int *gh);

/* Build pyramid levels 1..levels-1 of pyr (a host array of device planes) from
 * level 0 (Section II-B).  Enqueued on `stream`.
 * Errors: FAST_EINVAL (see fast_plane; level sizes must be floor halvings). */
int fast_pyr_build(fast_ctx *ctx, const fast_plane *pyr, int levels, void *stream);

/* Plain path, one frame: the detector of Sections II-B to II-D and Algorithm 1
 * (pyramid, FAST segment test and score with Eq. (1), 3x3 NMS, the per-cell
 * maximum over all levels).  Builds levels 1..levels-1 into pyr[1..] and writes
 * one fast_feature per grid cell into `out` (device, gw*gh slots, row-major).
 * Everything is enqueued on `stream`; no host synchronisation.
 * Errors: FAST_EINVAL for null pointers, levels not in 1..8, t not in 0..255,
 * n not in 1..16, cell < 1 or cell > 256 or cell % 2^(levels-1) != 0, a plane
 * that breaks the fast_plane rules, level sizes other than floor halvings;
 * FAST_EHIP if a launch fails. */
int fast_detect_grid(fast_ctx *ctx, const fast_plane *pyr, int levels, int t, int n,
                     int cell, fast_feature *out, void *stream);

/* fast_detect_grid with a corner score kind (FAST_SCORE_*; Section II-D).
 * fast_detect_grid is this call with FAST_SCORE_SADB.
 * Errors: as fast_detect_grid, and FAST_EINVAL for an unknown score kind. */
int fast_detect_grid_score(fast_ctx *ctx, const fast_plane *pyr, int levels, int t, int n,
                           int cell, int score, fast_feature *out, void *stream);

/* The score stage alone (Section II-D): build levels 1..levels-1 into pyr[1..]
 * as fast_detect_grid does, and write every level's corner scores of kind
 * `score` (FAST_SCORE_*; 0 in the 3-pixel border and where the segment test
 * fails) to maps[k], a device array of pyr[k].height rows of map_pitch[k]
 * uint16 elements (map_pitch[k] >= pyr[k].width, maps 2-byte aligned;
 * elements past the width are not written).  maps and map_pitch are host
 * arrays of `levels` entries.  Enqueued on `stream`.
 * Errors: as fast_detect_grid_score, and FAST_EINVAL for a NULL or misaligned
 * map or a pitch below the level width. */
int fast_score_maps(fast_ctx *ctx, const fast_plane *pyr, int levels, int t, int n, int score,
                    uint16_t *const *maps, const int32_t *map_pitch, void *stream);

/* Standalone non-maxima suppression over the (2 radius + 1)^2 Moore
 * neighbourhood (Section I-B; radius 1..4, the paper's n) and the cell
 * arg-max across levels (Sections II-B, II-C), from score maps laid out as
 * fast_score_maps writes them for a level-0 size of width x height (level k
 * is the floor halving k times).  Same tie rules and output slots as
 * fast_detect_grid; with radius 1 the slots equal fast_detect_grid's.
 * Errors: FAST_EINVAL for levels not in 1..8, sizes not in 1..65535, radius
 * not in 1..4, a cell rule violation (as fast_detect_grid), NULL out, or a bad
 * map (as fast_score_maps); FAST_EHIP if the launch fails. */
int fast_nms_grid(fast_ctx *ctx, uint16_t *const *maps, const int32_t *map_pitch, int width,
                  int height, int levels, int radius, int cell, fast_feature *out, void *stream);

/* Lucas-Kanade feature tracking (Section II-E): the pyramidal, approximated
 * simultaneous inverse compositional tracker with a translational warp
 * W(x, t) = x + t and affine illumination, q = (tx, ty, alpha, beta).  Each
 * feature's patch (16x16 on levels 0-1, 8x8 above, at p + (i - S/2, j - S/2))
 * of the template pyramid `tpl` is aligned to the current pyramid `img`,
 * coarse to fine; U(x) = [(1+alpha) dT/dx, (1+alpha) dT/dy, T, 1] and the
 * Hessian sum U U^T are formed once per level at the alpha it starts with,
 * and each iteration solves H dq = sum U [I(x+t) - (1+alpha) T - beta] and
 * applies t -= dt, alpha += dalpha, beta += dbeta.  Samples are bilinear,
 * template gradients central differences.  fp32 on the device.
 * tpl, img:  `levels` device planes each (as fast_detect_grid), equal sizes.
 * feats:     device, nfeat x 2 floats: (x, y) in level-0 pixels of tpl.
 * q:         device, nfeat x 4 floats: in, the initial (tx, ty, alpha, beta)
 *            with t in level-0 pixels; out, the estimate.
 * status:    device, nfeat int32: FAST_TRACK_* below.
 * iters:     device, nfeat int32 iterations over all levels, or NULL.
 * mode:      FAST_TRACK_GAIN | FAST_TRACK_OFFSET bits select alpha and beta
 *            (translation is always estimated; unselected ones keep q's).
 * max_iter:  iterations per level, 0..1000; eps: a level stops once
 *            |delta t| < eps level pixels (eps >= 0).
 * A level-k feature sits at (x, y) / 2^k and the level-k translation is
 * t / 2^k.  A track is lost when a template patch with its 1-pixel gradient
 * margin does not fit a level, when the warped patch leaves the level, or
 * when a Cholesky pivot of the Hessian falls to 1e-6 of its diagonal entry.
 * feats, q, status and iters must be 4-byte aligned.
 * Errors: FAST_EINVAL for bad planes, mismatched sizes, bad mode, max_iter,
 * eps or nfeat (< 0 or > 2^24), NULL arrays with nfeat > 0, or misaligned
 * arrays; FAST_EHIP if the launch fails.  Asynchronous on `stream`; nfeat = 0
 * enqueues nothing. */
#define FAST_TRACK_GAIN 1
#define FAST_TRACK_OFFSET 2
#define FAST_TRACK_OK 0
#define FAST_TRACK_TEMPLATE_OUTSIDE 1
#define FAST_TRACK_LOST_OUTSIDE 2
#define FAST_TRACK_SINGULAR 3
int fast_track(fast_ctx *ctx, const fast_plane *tpl, const fast_plane *img, int levels,
               const float *feats, float *q, int32_t *status, int32_t *iters, int nfeat, int mode,
               int max_iter, float eps, void *stream);

/* The detect-and-track loop of the paper's tracker evaluation (Section III-D)
 * for many camera streams in one call, with every feature list resident in
 * device memory, so a frame needs no host round trip.  One job is one
 * stream's step from its previous frame to the current one:
 *   1. track the stream's live features (fast_track, from a zero initial
 *      estimate; the live count is read from device memory);
 *   2. keep the tracked ones (status FAST_TRACK_OK), in order, moved by their
 *      estimated translation, and drop the rest;
 *   3. when fewer than redetect_below remain, mark the cells that hold a kept
 *      feature (cell of a level-0 position p: floor(p / cell), row-major) and
 *      append the strongest winners of the other cells of this frame's
 *      detection (score descending, then cell index ascending) at their
 *      level-0 positions (x << level, y << level), up to the capacity.  Which
 *      features a re-detection adds is not stated in the paper; this is the
 *      reading taken.
 * The caller detects on the current frame first (fast_submit or
 * fast_detect_grid_score, which also builds the current pyramid's levels),
 * on the same stream.  The paper's evaluation detects with SAD-A.
 * tracking parameters (mode, max_iter, eps) are as for fast_track and shared
 * by all jobs.  Asynchronous on `stream`; the job table travels in one copy
 * from a context staging slot, like fast_submit (FAST_EBUSY when all are in
 * flight); *ticket (may be NULL) works as for fast_submit.
 * Errors: FAST_EINVAL for NULL jobs, njobs not in 1..FAST_MAX_JOBS, bad
 * tracking parameters, or a job with bad planes (as fast_track; prev and cur
 * of equal sizes), a cell rule violation, more than FAST_MAX_GRID_CELLS
 * cells, NULL or misaligned (4 bytes) device arrays, capacity not in
 * 1..FAST_MAX_TRACKS or redetect_below not in 0..capacity; nothing is then
 * enqueued. */
#define FAST_MAX_TRACKS 1024
#define FAST_MAX_GRID_CELLS 65536
typedef struct {
    const fast_plane *prev;      /* host array of `levels` planes: the previous frame's pyramid,
                                    or NULL on the stream's first frame (nothing is tracked) */
    const fast_plane *cur;       /* host array of `levels` planes: this frame's pyramid, levels built */
    int32_t levels;
    const fast_feature *slots;   /* device: this frame's cell winners, gw*gh for cur[0]'s size and cell */
    int32_t cell;
    int32_t capacity;            /* target track count, 1..FAST_MAX_TRACKS */
    int32_t redetect_below;      /* re-detect when fewer live tracks remain, 0..capacity */
    float *feats;                /* device, capacity x 2: live features, level-0 (x, y); in and out */
    int32_t *count;              /* device, 1: live features in feats; in and out */
    float *q;                    /* device, capacity x 4: scratch (tracking estimates) */
    int32_t *status;             /* device, capacity: scratch (tracking statuses) */
    int32_t *info;               /* device, 4: out (tracked, re-detected 0/1, live, 0) */
} fast_frontend_job;
int fast_frontend_step(fast_ctx *ctx, const fast_frontend_job *jobs, int njobs, int mode, int max_iter,
                       float eps, void *stream, uint64_t *ticket);

/* Batched path: all `njobs` requests (1..FAST_MAX_JOBS, any mix of sizes and
 * parameters) run in one persistent launch fed by a device-side work queue.
 * The job table and its work-item list are enqueued on `stream` as one copy
 * from library-owned pinned memory, followed by the kernels; nothing blocks.
 * *ticket identifies the submission for fast_poll / fast_wait.
 * Each job is validated like fast_detect_grid; one bad job rejects the whole
 * submission with FAST_EINVAL and nothing is enqueued.  FAST_EBUSY if the
 * context's in-flight table slots are all taken by unfinished submissions. */
int fast_submit(fast_ctx *ctx, const fast_job *jobs, int njobs, void *stream,
                uint64_t *ticket);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): fast_submit
 * without any allocation.  The queue counters, job table and work items go
 * to a fixed scratch array in device memory that the library holds on each
 * device from the first fast_ctx_create there until the process ends
 * (FAST_STATIC_SCRATCH_BYTES, about 336 KiB), through a pinned staging buffer
 * the context set up at creation; the call then enqueues the same kernels as
 * fast_submit.  The caller still owns every plane and output.
 * Limits: njobs <= FAST_STATIC_MAX_JOBS and at most FAST_STATIC_MAX_ITEMS
 * work items (regions of the default 64-pixel side, counted once more for
 * jobs of more than 3 levels); beyond either, FAST_EINVAL and nothing is
 * enqueued.
 * The scratch is shared by every context and stream on the device and keeps
 * the last call's contents (the counters are rewritten as zeros by each
 * call): calls whose work overlaps on one device race.  Calls on one stream
 * are ordered.  A call waits for the previous call's table copy to leave the
 * staging buffer before it rewrites it.
 * ticket may be NULL (no completion event); otherwise it works as for
 * fast_submit.  Errors: as fast_submit, except FAST_EBUSY and FAST_ENOMEM,
 * which it never returns. */
#define FAST_STATIC_MAX_JOBS 256
#define FAST_STATIC_MAX_ITEMS 32768
#define FAST_STATIC_SCRATCH_BYTES 344320
int fast_submit_static(fast_ctx *ctx, const fast_job *jobs, int njobs, void *stream,
                       uint64_t *ticket);

/* 1 if the submission has finished, 0 if still pending; never blocks.
 * Errors: FAST_EINVAL for an unknown ticket, FAST_EHIP for a device error. */
int fast_poll(fast_ctx *ctx, uint64_t ticket);

/* Block until the submission finishes or timeout_ms passes (timeout_ms < 0:
 * no limit).  Polls without sleeping for the first 2 ms, then every 20 us.
 * Returns FAST_OK, FAST_ETIMEDOUT, or an error. */
int fast_wait(fast_ctx *ctx, uint64_t ticket, int timeout_ms);

/* A resident batch: the job table is uploaded once into context-owned device
 * memory; each launch re-runs the whole batch on the frames currently in the
 * jobs' planes.  flags = 0: every launch enqueues the kernels directly from the
 * resident table, with the context's launch shape at that moment.
 * flags = FAST_PLAN_GRAPH: the launch sequence (with the launch shape current
 * at creation) is captured into a HIP graph, and every launch replays it.
 * *plan_id receives a handle (>= 0).  Launches of one plan share its
 * work-queue counter, so they must not run concurrently (enqueue them on one
 * stream).  Errors as for fast_submit, FAST_EINVAL for unknown flags,
 * FAST_ENOMEM. */
#define FAST_PLAN_GRAPH 1
int fast_plan_create(fast_ctx *ctx, const fast_job *jobs, int njobs, int flags, int *plan_id);

/* Launch a resident batch on `stream`.  If ticket is non-NULL, a completion
 * event is recorded and *ticket works as for fast_submit; with ticket = NULL
 * no event is recorded (the caller synchronises on the stream itself). */
int fast_plan_launch(fast_ctx *ctx, int plan_id, void *stream, uint64_t *ticket);

/* Release a resident batch.  Never waits: the plan's device memory and graph
 * are freed once the launches already enqueued have completed (at a later
 * fast_plan_create, or in fast_ctx_destroy).  The stream of the plan's last
 * launch must still exist when this is called. */
int fast_plan_destroy(fast_ctx *ctx, int plan_id);

/* Launch-shape tuning (the autotuner's knobs), per context.
 * region: side of the square region one workgroup owns, in level-0 pixels,
 *         rounded up to a multiple of the cell (16..256), for every entry
 *         point; 0 restores the default of a new context: 64, except that
 *         a one-frame call (fast_detect_grid*, fast_score_maps,
 *         fast_nms_grid) on a frame of at most 3 levels with fewer 64-pixel
 *         regions than half the compute units uses 32 (faster there);
 * block:  threads per workgroup, a multiple of 64 in 64..512;
 * persistent_blocks_per_cu: workgroups per compute unit for the persistent
 *         batched kernel (1..16).
 * Errors: FAST_EINVAL for values out of range. */
int fast_set_launch(fast_ctx *ctx, int region, int block, int persistent_blocks_per_cu);

/* Tuned region sides for one-frame calls (the autotuner's table, keyed by
 * frame shape).  An entry applies to fast_detect_grid*, fast_score_maps and
 * fast_nms_grid calls on a frame of exactly its width, height, levels and
 * cell; region is then the side of the square region one workgroup owns, in
 * level-0 pixels, rounded as for fast_set_launch.  Shapes without an entry
 * keep the default rule, and a nonzero region set with fast_set_launch
 * overrides the table.  Batched submissions are not affected (they use the
 * fast_set_launch shape).  The table is copied; n = 0 clears it.
 * Errors: FAST_EINVAL for n not in 0..FAST_MAX_SHAPES, NULL entries with
 * n > 0, an entry with bad sizes, levels or cell (as fast_detect_grid), a
 * region not in 16..256, or a shape listed twice (the table is then left as
 * it was). */
typedef struct {
    int32_t width, height, levels, cell;
    int32_t region;
} fast_shape_region;
#define FAST_MAX_SHAPES 1024
int fast_set_shape_table(fast_ctx *ctx, const fast_shape_region *entries, int n);

/* The region side, in level-0 pixels after rounding to whole cells, that a
 * one-frame call on a frame of this shape uses with the context's current
 * settings (an explicit fast_set_launch side, the shape table, or the
 * default rule).  Errors: FAST_EINVAL for NULL region or arguments that
 * fast_detect_grid would reject. */
int fast_shape_region_of(fast_ctx *ctx, int width, int height, int levels, int cell, int *region);

/* Native serving loop (not in the paper; the continuous-batching server of
 * camera streams).  fast_pump_run replays a schedule of frame arrivals by the
 * host clock and serves them: whenever a launch lane is free, the oldest
 * arrived frames whose stream has a free result slot form the next launch
 * (up to max_batch frames through fast_submit when `batched`, else one frame
 * through fast_detect_grid_score), the results are copied to the slots' host
 * buffers, and an event marks the launch done.  The loop busy-polls; nothing
 * crosses to Python until every request is served.
 *
 * A stream describes its resident frames and result slots (all memory
 * caller-owned; device pointers unless noted): */
typedef struct {
    int32_t levels, t, n, cell, score;   /* detector parameters (as fast_job) */
    int32_t pool_frames;                 /* P >= 1 */
    const fast_plane *pool;              /* host array of P level-0 planes: frame k of the stream
                                            is pool[k % P] */
    int32_t slots;                       /* S >= 1: results in flight at once for this stream */
    const fast_plane *upper;             /* host array of S * (levels-1) planes: slot s builds
                                            levels 1.. into upper[s*(levels-1) ..] */
    fast_feature *const *out;            /* host array of S device grids (gw*gh slots each) */
    void *const *host_out;               /* host array of S pinned host buffers of gw*gh*8 bytes
                                            that receive each result, or NULL (no copy) */
} fast_pump_stream;

typedef struct {
    int32_t stream;      /* index into the streams array */
    int32_t frame;       /* frame index k (served from pool[k % P]) */
    double arrival_s;    /* arrival time in seconds after the run starts, non-decreasing */
} fast_pump_request;

#define FAST_PUMP_MAX_LANES 8
/* Serve `nreq` requests with `lanes` (1..FAST_PUMP_MAX_LANES) launches in
 * flight.  Outputs, per request (host arrays of nreq): done_s, the time the
 * loop saw its launch complete (seconds after the start), and slot_of, the
 * result slot it used; *nbatches receives the number of launches.  The run
 * gives up after max_seconds of wall time (FAST_ETIMEDOUT, with every launch
 * drained).  Errors: FAST_EINVAL for NULL arrays, nreq < 1, a request naming
 * no stream, decreasing arrivals, lanes or max_batch out of range, or a
 * stream or slot that fast_submit would reject; FAST_EHIP if a launch fails
 * (every lane is drained before returning).  Uses the context's job tables
 * like fast_submit, so no other submission may be in flight on it. */
int fast_pump_run(fast_ctx *ctx, const fast_pump_stream *streams, int nstreams, const fast_pump_request *reqs,
                  int nreq, int lanes, int max_batch, int batched, double max_seconds, double *done_s,
                  int32_t *slot_of, int32_t *nbatches);

/* The same loop serving the detect-and-track front end (fast_frontend_step)
 * of every stream: a stream's frames are served in order, one at a time.  A
 * launch detects (SAD-A) the frames of its streams into their current
 * pyramids and cell grids (one fast_submit), runs one fast_frontend_step for
 * them from each stream's previous frame, and copies each step's info to
 * info_host.  The two pyramids of a stream alternate; level 0 is the pool
 * frame.  `streams` gives levels, t, n, cell and the pool (slots must be at
 * least 1; upper, out and host_out are not used); fe[i] holds stream i's
 * state (device memory unless noted).  A launch holds two of the context's
 * job tables, so lanes is at most FAST_PUMP_MAX_LANES / 2. */
typedef struct {
    const fast_plane *upper;   /* host array of 2 * (levels-1) planes: levels 1.. of pyramid 0, then 1 */
    fast_feature *grid;        /* this frame's cell winners */
    float *feats;              /* capacity x 2, live features; in and out across frames */
    int32_t *count;            /* 1: live features (0 before the stream's first frame) */
    float *q;                  /* capacity x 4, scratch */
    int32_t *status;           /* capacity, scratch */
    int32_t *info;             /* 4: (tracked, re-detected, live, 0) of the last step */
    void *info_host;           /* pinned host copy of info after each step, or NULL */
    int32_t capacity;          /* 1..FAST_MAX_TRACKS */
    int32_t redetect_below;    /* 0..capacity */
} fast_pump_frontend;
/* Errors as fast_pump_run, plus those of fast_frontend_step. */
int fast_pump_run_frontend(fast_ctx *ctx, const fast_pump_stream *streams, const fast_pump_frontend *fe,
                           int nstreams, const fast_pump_request *reqs, int nreq, int lanes, int max_batch,
                           int mode, int max_iter, float eps, double max_seconds, double *done_s,
                           int32_t *nbatches);

#ifdef __cplusplus
}
#endif
#endif
