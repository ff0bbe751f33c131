// Internal declarations shared by the kernels and the host runtime of
// libfastgrid.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastgrid.h"

// Device-side description of one detection job (one frame).
struct fg_job {
    uint8_t *lvl[FAST_MAX_LEVELS];   // level planes; [0] is the input
    int32_t w[FAST_MAX_LEVELS];
    int32_t h[FAST_MAX_LEVELS];
    int32_t pitch[FAST_MAX_LEVELS];
    int32_t levels, t, n, cell;
    int32_t score;                   // corner score kind (FAST_SCORE_*)
    uint16_t *smap[FAST_MAX_LEVELS]; // score maps (score-map and standalone-NMS entry points)
    int32_t smap_pitch[FAST_MAX_LEVELS];   // their pitches in elements
    fast_feature *out;               // gw*gh slots
    int32_t gw, gh;                  // grid size in cells
    int32_t rcells;                  // cells per region side
    int32_t rx, ry;                  // regions across, down
    int32_t region_base;             // first work item of this job in a batch
};

// Launch shape knobs (set per context by fast_set_launch / the autotuner).
struct fg_launch {
    int region;          // target region side in level-0 pixels, batches
    int plain_region;    // the same for one-frame calls; 0 = chosen per frame
    int block;           // threads per workgroup
    int blocks_per_cu;   // persistent kernel occupancy target
    int num_cu;          // compute units on the device
};

// Dynamic LDS bytes of the detect kernels for a workgroup size.
size_t fg_smem_bytes(int block);

// Fill the derived fields of a job (grid, regions) for a launch shape.
void fg_job_layout(fg_job &j, const fg_launch &L);

// Lucas-Kanade tracking of nfeat features, one wave64 each.
struct fg_track_args {
    const uint8_t *tpl[FAST_MAX_LEVELS];
    const uint8_t *img[FAST_MAX_LEVELS];
    int32_t w[FAST_MAX_LEVELS], h[FAST_MAX_LEVELS];
    int32_t tpitch[FAST_MAX_LEVELS], ipitch[FAST_MAX_LEVELS];
    int32_t levels;
    const float *feats;   // nfeat x (x, y)
    float *q;             // nfeat x (tx, ty, alpha, beta), in and out
    int32_t *status;
    int32_t *iters;       // or null
    int32_t nfeat, mode, max_iter;
    float eps;
};
hipError_t fg_launch_track(const fg_track_args &A, hipStream_t s);

// One camera stream's step of the detect-and-track loop (fast_frontend_step):
// tracking arguments (tpl = previous pyramid, img = current; feats, q and
// status hold `capacity` entries; nfeat unused: the live count is *count),
// this frame's cell winners, and the selection rule.
struct fg_fe_job {
    fg_track_args A;
    const fast_feature *slots;   // gw*gh cell winners of the current frame
    int32_t *count;              // live features: in, tracked from the previous frame; out, after the step
    int32_t *info;               // out: tracked, re-detected (0/1), live, 0
    int32_t cell, gw, gh;
    int32_t capacity;            // the target track count
    int32_t redetect_below;      // re-detect when fewer live tracks remain
    int32_t has_prev;            // 0 on a stream's first frame: nothing to track
    int32_t feat_base;           // first wave of this job in the tracking launch
};

// Tracking of every job's live features (one wave per feature slot, total_slots
// = sum of capacities), then the update of every job's feature list.
hipError_t fg_launch_frontend(const fg_fe_job *jobs_dev, int njobs, int total_slots, hipStream_t s);

// Plain path: one frame.  Enqueues the pyramid (levels 1..L-1) and detection.
hipError_t fg_launch_plain(const fg_job &j, const fg_launch &L, hipStream_t s);

// Pyramid only, one frame.
hipError_t fg_launch_pyramid(const fg_job &j, hipStream_t s);

// One frame's score maps (j.smap): builds levels 1.. like fg_launch_plain and
// writes every level's scores instead of selecting features.
hipError_t fg_launch_score_maps(const fg_job &j, const fg_launch &L, hipStream_t s);

// Standalone NMS over (2 radius + 1)^2 neighbourhoods and the cell arg-max
// from j.smap (j.lvl unused) into j.out.
hipError_t fg_launch_nms_grid(const fg_job &j, int radius, hipStream_t s);

// The persistent batched kernels' counter buffer: FG_QUEUES work queues, the
// head of queue c at word FG_QUEUE_STRIDE * c, and the exit count at word
// FG_QUEUES * FG_QUEUE_STRIDE.  The heads sit 256 bytes apart, on separate
// cache lines: one shared head serialises every ticket of a launch (about
// 13 ns each on MI355X, which alone bounded the 64-frame batch near 100 us).
constexpr int FG_QUEUES = 8;
constexpr int FG_QUEUE_STRIDE = 64;
constexpr int FG_EXIT_WORD = FG_QUEUES * FG_QUEUE_STRIDE;
constexpr int FG_COUNTER_WORDS = FG_EXIT_WORD + FG_QUEUE_STRIDE;
// Consecutive work items a queue hands out before the next queue's run: 16
// neighbouring 64x64 regions on one XCD cut the batch's fetched bytes 3x
// against runs of one; runs of 64 cut them further but leave the queues
// (and XCDs) finishing up to 2% apart.
constexpr int FG_QUEUE_RUN = 16;

// One work item of the batched kernel: a region of a job.
struct fg_item {
    uint32_t job;
    uint32_t region;
};

// Pyramid levels detected from one level-0 load; deeper levels take a second
// pass.
constexpr int FG_MAX_FUSED = 3;

// Batched path: `jobs_dev` is a device copy of njobs jobs whose region_base
// fields are prefix sums.  items[0 .. total) lists every region of every job
// once, in any order; items[total .. total + total_upper) lists every region
// of the jobs with more than FG_MAX_FUSED levels (their deeper levels).
// all_single: every job's regions are single 64x64 sub-tiles (the pipelined
// kernel applies).  `counter` holds FG_COUNTER_WORDS zero-initialised words
// that the kernel re-arms itself on exit.
hipError_t fg_launch_batch(const fg_job *jobs_dev, const fg_item *items, int njobs, int total,
                           int total_upper, int max_levels, int max_w1, int max_h1, bool all_single,
                           unsigned *counter, const fg_launch &L, hipStream_t s);

// Regions of at most this side (level-0 pixels) are one fused sub-tile.
constexpr int FG_SUB = 64;
